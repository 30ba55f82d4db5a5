// Host/device structures and launchers of the Navier-Stokes step kernels.
#pragma once

#include "wl_internal.h"

namespace wl {

// A velocity field with its boundary description (device pointers).  u[c]
// are interior face arrays; uout is the outflow plane (upper x boundary face)
// or null when there is none.
template <typename T>
struct VelField {
    const T* u[3];
    const T* uout;
    Grid g;
    int bclo[3], bchi[3];
    T U[3];
};

template <typename T>
struct BdimFields {
    const T* mu0[3];
    const T* mu1n[9];
    // Tile class per block of the cell tiling (launch_for): 0 where every
    // face of the tile has mu0 = 1 and mu1 n = 0, so BDIM is the identity
    // there; null treats every tile as touching the body.
    const unsigned char* cls = nullptr;
    // Per cell: 1 where the blend differs from f on any face of the cell
    // (mu0 != 1 or a nonzero mu1 n component); null: every cell.
    const unsigned char* cflag = nullptr;
};

template <typename T>
struct ProjCoeffs {
    const T* L[3];
    T Lc;
    // optional block classes of the fine level's launch_for tiling (see
    // Coeffs::cls): a class-0 block has every face Lc or 0 on a domain wall,
    // so all its cells are active
    const unsigned char* cls = nullptr;
};

template <typename T>
struct MeasureOut {
    T* mu0[3];
    T* mu1n[9];
    T* L[3];
    double* L64[3];  // optional FP64 copy of L (mixed-precision solves)
};

// Tile decomposition of a z-marching kernel: tiles_x * tiles_y columns of
// tile_x * tile_y cells, each split into chunks of zc planes.
struct TileMap {
    int tiles_x, tiles_y, nchunks, zc;
    unsigned nblocks;
    int remap;  // 1: XCD-contiguous block order (nblocks divisible by 8)
};
TileMap tile_map(const Grid& g, int tile_x, int tile_y, int zc);
int momentum_zchunk(const Grid& g, int per_cu);

struct BodyDev {
    int kind;
    double centre[3];
    double radius;
    double eps;
    double radius2;   // torus tube radius (kind 2)
};

// Rigid motion of a body at one time, for the BDIM blend: the body velocity
// V_b(x) = xdot + w x (x - X) and its gradient dV_b,i/dx_j = eps_ikj w_k.
// on = 0: body at rest (V_b = 0).
struct BodyMotionDev {
    int on;
    double X[3], xdot[3], w[3];
};

template <typename T>
wl_status ns_measure(const Grid& g, const BodyDev& body, const int bclo[3], const MeasureOut<T>& M,
                     hipStream_t s);
template <typename T>
wl_status ns_momentum(const VelField<T>& E, const T* const un[3], T* const f[3], T nu, bool corr,
                      bool allper, const double* dt_dev, hipStream_t s);
// Corrector convection-diffusion of a periodic FP32 3D grid with uniform
// coefficients Lc whose predictor projection was not stored: E holds the
// predictor stage field u* and p its pressure; the kernel uses
// u1 = u* - dt Lc grad(p) (same rounding as ns_project).
wl_status ns_momentum_proj(const VelField<float>& E, const float* const un[3], float* const f[3],
                           float nu, const double* dt_dev, const float* p, float Lc,
                           hipStream_t s);
// Convective outflow plane and its exit-flux balance; part: scratch for two
// FP64 sums per 256 plane cells (a simulation's reduction partials, free
// between the momentum kernel and the divergence).
template <typename T>
wl_status ns_outflow(const Grid& g, const T* ue_x, const T* out_e, const T* out_n, const T* f_x,
                     T Ux, bool corr, const double* dt_dev, T* fout, double* part,
                     hipStream_t s);
template <typename T>
wl_status ns_bdim(const VelField<T>& F, const BdimFields<T>& B, T* const out[3], hipStream_t s,
                  const BodyMotionDev& motion = BodyMotionDev{});
// The same blend left in f itself (f = the arrays of F): only the cells whose
// blend differs from f (B.cflag) are touched, through the scratch arrays w;
// f serves as u* unchanged elsewhere.  Needs B.cflag.
template <typename T>
wl_status ns_bdim_in_place(const VelField<T>& F, T* const f[3], const BdimFields<T>& B,
                           T* const w[3], hipStream_t s,
                           const BodyMotionDev& motion = BodyMotionDev{});
// Tile classes (see BdimFields::cls) from the measured mu0 / mu1 n.
// With cflag, also the per-cell flags (see BdimFields::cflag).
template <typename T>
wl_status ns_tile_class(const Grid& g, const BdimFields<T>& B, unsigned char* cls, hipStream_t s,
                        unsigned char* cflag = nullptr);
// p_check (periodic, uniform, 3D): also the first residual check of the
// pressure solve that starts from p, with Poisson coefficient Lp (partials of
// [sigma, sigma^2, c, c^2], c = sigma - A p; see k_divergence).
// *nslots (if given): the partial slots written (workgroups of the launch).
template <typename T>
wl_status ns_divergence(const VelField<T>& V, const ProjCoeffs<T>& C, bool unif, double c,
                        const double* dt_dev, T* sigma, double* partial, bool allper,
                        hipStream_t s, const T* p_check = nullptr, T Lp = T(0),
                        size_t* nslots = nullptr);
// Workgroups of the tiled divergence-with-check kernel on g (nblocks 0 when
// it does not apply); partial slot capacity must cover them.
TileMap div_check_map(const Grid& g);
template <typename T>
wl_status ns_project(const VelField<T>& V, const T* p, const ProjCoeffs<T>& C, bool unif, double c,
                     const double* dt_dev, T* const out[3], bool cfl, double* partial, bool allper,
                     hipStream_t s);
template <typename T>
wl_status ns_cfl(const VelField<T>& V, bool allper, double* partial, hipStream_t s);
// post (may be null): also post dt to the host mailbox (the caller then
// calls host_posted).
wl_status ns_dt_from_max(const double* partial, size_t nslots, double cfl, double visc,
                         double* dt_dev, double* max_dev, hipStream_t s,
                         const MailboxPost* post = nullptr);
wl_status ns_set_scalar(double* p, double v, hipStream_t s);
template <typename T>
wl_status ns_init_velocity(const Grid& g, const int bclo[3], const double U[3], T* const u[3],
                           hipStream_t s);

}  // namespace wl
