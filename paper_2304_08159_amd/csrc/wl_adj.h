// Adjoint (reverse-mode) kernels of the Navier-Stokes step and of the drag
// functional.  The derivation is written next to each kernel in adjoint.hip.
#pragma once

#include "wl_ns.h"

namespace wl {

// Padded adjoint array: every velocity component gets two ghost layers per
// side (none along z in 2D), indexed (i+2) + P0 ((j+2) + P1 (k+o2)).
struct PadGrid {
    int P0, P1, P2, o2;
};
PadGrid pad_grid(const Grid& g);
inline size_t pad_cells(const PadGrid& p) { return size_t(p.P0) * p.P1 * p.P2; }

template <typename T>
struct PadField {
    T* a[3];
    PadGrid pg;
};

// Pointer bundles passed by value to the kernels.
template <typename T>
struct AdjPtrs {
    T* p[3];
};
template <typename T>
struct AdjPtrs9 {
    T* p[9];
};

// R'(e)^T Rbar gathered on the padded grid (e: the stage's evaluation field).
template <typename T>
wl_status adj_flux(const VelField<T>& E, T* const Rbar[3], T nu, const PadField<T>& out, bool allper,
                   hipStream_t s);
// BDIM^T gbar gathered on the padded grid.
template <typename T>
wl_status adj_bdim(const Grid& g, T* const gbar[3], T* const mu0[3], T* const mu1n[9],
                   const PadField<T>& out, hipStream_t s);
// mu0bar += f gbar, mu1nbar_cj += (f(K+dj) - f(K-dj))/2 gbar on interior faces.
template <typename T>
wl_status adj_bdim_param(const VelField<T>& F, T* const gbar[3], T* const mu0b[3], T* const mu1nb[9],
                         hipStream_t s);
// acc_c += fold(pad_c) on stored faces (interior faces only); acc_out += the
// outflow-plane ghosts of the x component.
template <typename T>
wl_status adj_fold(const VelField<T>& geom, const PadField<T>& pad, T* const acc[3], T* acc_out,
                   hipStream_t s);
// rhs = pbar + coef * div(L ubar)   (cells; pbar may be null)
template <typename T>
wl_status adj_proj_rhs(const Grid& g, const T* pbar, T* const ubar[3], T* const L[3], T Lc, bool unif,
                       double coef, T* rhs, hipStream_t s);
// gbar_d = ubar_d + (sbar(K - d) - sbar(K)) / coef on interior faces (0 on
// boundary faces); Lbar_d += (G p)_d ((G sbar)_d - coef ubar_d).
template <typename T>
wl_status adj_proj_update(const Grid& g, T* const ubar[3], const T* sbar, const T* p, T* const L[3],
                          T Lc, bool unif, double coef, T* const gbar[3], T* const Lbar[3],
                          hipStream_t s);
// outflow plane: gout = fout_bar + uout_bar + sbar(n0-1)/coef, then fout_bar = gout - mean(gout).
template <typename T>
wl_status adj_plane_proj(const Grid& g, const T* uoutb, const T* sbar, double coef, T* foutb,
                         hipStream_t s);
// Stage terms of the outflow plane: base_bar += wb * fout_bar; eout_bar +=
// -U a dt fout_bar; e_x(n0-1) bar += U a dt fout_bar.
template <typename T>
wl_status adj_plane_stage(const Grid& g, const T* foutb, double wb, double adt, T Ux, T* baseb,
                          T* eoutb, T* ebx, hipStream_t s);
// y = alpha x (+ y if accumulate) on interior faces; boundary faces set to 0.
template <typename T>
wl_status adj_faces_axpy(const Grid& g, T* const x[3], double alpha, T* const y[3], bool accumulate,
                         hipStream_t s);
// y += x over n cells.
template <typename T>
wl_status adj_cells_add(size_t n, const T* x, T* y, hipStream_t s);
// Geometry adjoints -> parameter gradient (r, cx, cy, cz): partial sums per
// block into partial[4*blk + k]; the accumulators are cleared.
template <typename T>
wl_status adj_params(const Grid& g, const BodyDev& body, T* const Lb[3], T* const mu0b[3],
                     T* const mu1nb[9], double* partial, hipStream_t s);
// Drag of the current pressure: partial sums of (w, p, p w, active) with
// w = n_x K(d) at cell centres.
template <typename T>
wl_status drag_sums(const Grid& g, const BodyDev& body, const T* p, T* const L[3], double* partial,
                    hipStream_t s);
// pbar = -weight (w - wmean) on active cells (0 elsewhere) and partial sums of
// -weight (p - pmean) dw/dtheta_k (4 per block).
template <typename T>
wl_status drag_adj(const Grid& g, const BodyDev& body, const T* p, T* const L[3], double weight,
                   const double* means /* device: [wmean, pmean] */, T* pbar, double* partial,
                   hipStream_t s);
wl_status reduce_cols(const double* partial, size_t nslots, int ncomp, double* out, hipStream_t s);

}  // namespace wl
