// Internals of liblbm.so shared by the forward (lbm_api.hip) and adjoint
// (lbm_adjoint.hip) translation units: workspace layout and the handle.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>

#include "lbm.h"
#include "lbm_device.hpp"

namespace lbmi {

constexpr int kRedBlocks = 1024;  // partial sums of the first reduction pass
constexpr int kRedThreads = 256;
constexpr int kStatSlots = 16;    // doubles per partial / in the result

struct Layout {
    size_t fA, fB, rA, rB, nbr, wet, mrho, mu, uxprev, partial, dstats, conv_part;
    // fluid-only layout: neighbour table [Q-1][T], density / psi / U of the
    // listed nodes [n_comp][T], lattice index of each listed node [T], list
    // index of each lattice node [N] (T = N rounded up to 64)
    size_t ftab, frho, fpsi, fU, fdmap, femap;
    size_t total;
};

inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }
inline int q_of(int lat) { return lat == LBM_D2Q9 ? 9 : 19; }
inline size_t store_bytes(int st) {
    return st == LBM_STORE_F64 ? 8 : ((st == LBM_STORE_F32 || st == LBM_STORE_F32_F64) ? 4 : 2);
}
inline size_t real_bytes(int st) { return (st == LBM_STORE_F64 || st == LBM_STORE_F32_F64) ? 8 : 4; }
inline bool is_dev(int st) { return st == LBM_STORE_F16DEV || st == LBM_STORE_BF16DEV; }

// Explicit population buffers for one launch of the fused step.
struct Buffers {
    const void* fin;
    void* fout;
    const float* rin;
    float* rout;
};

}  // namespace lbmi

struct lbm_handle {
    lbm_params p;
    lbmi::Layout lay;
    hipStream_t stream;
    char* ws;
    int N, NA, NB, NCc;
    int cur;          // 0: state in fA/rA, 1: state in fB/rB
    int64_t step;
    int64_t since_check;
    bool have_prev;
    bool wet_uniform;  // no per-node wetting field was given: p.wet[k] everywhere
    bool mostly_fluid; // under 10 % solid nodes: tiles carry even work
    bool has_res;      // the mask has reservoir nodes (open boundaries)
    // reservoir densities of the streaming that the next pull completes: the
    // pull of step t streams the populations of step t - 1, so a density set
    // between steps reaches the anti-bounce-back inflow one step later
    // (p.res_rho, the newest value, is what the force gather sees at once)
    double res_active[2][2];
    int conv_plane;    // plane of the convective outlet, -1: none
    int chunk_override;
    // fluid-only layout: ids [0, n_col) are the fluid nodes in lattice order,
    // [n_col, n_fl) the convective outlet's nodes (pulled from, not
    // collided), [n_fl, n_sol) the solid nodes with a fluid neighbour,
    // [n_sol, n_r1) and [n_r1, n_ext) the nodes of reservoirs 0 and 1; fl_T
    // is the row stride of the populations and the table (a multiple of 64);
    // [conv_lo, conv_hi) the fluid ids of the plane below the outlet
    int n_col, n_fl, n_sol, n_r1, n_ext, fl_T, conv_lo, conv_hi;
};

namespace lbmi {
// One fused step from b.fin to b.fout (the handle's own buffers are untouched).
hipError_t run_step_buffers(lbm_handle* h, const Buffers& b);
// Fluid-only layout (lbm_fluid.hip).  fluid_build lists the nodes and fills
// the neighbour table from the mask and the neighbour words already in the
// workspace (synchronises; returns an lbm_error code); fluid_init sets the
// populations to the equilibrium of device rho0 / u0 (lattice order, compute
// type); fluid_step runs one step from the current buffer into the other;
// fluid_moments writes lattice-order moments as the dense moment kernel does.
int fluid_build(lbm_handle* h);
hipError_t fluid_init(lbm_handle* h, const void* rho0, const void* u0);
hipError_t fluid_step(lbm_handle* h);
hipError_t fluid_moments(lbm_handle* h, int comp, void* rho, void* u);
// Convective outlet after a step of the fluid layout (before the swap).
hipError_t fluid_conv(lbm_handle* h);
// Pointer to the handle's current state buffer.
inline void* state_ptr(lbm_handle* h) { return h->ws + (h->cur ? h->lay.fB : h->lay.fA); }
// Kernel arguments of the handle's current step (bufs: explicit buffers).
template <class R>
inline void fill_args(lbm_handle* h, lbm::StepArgs<R>& a, const Buffers* bufs) {
    const lbm_params& p = h->p;
    std::memset(&a, 0, sizeof(a));
    char* ws = h->ws;
    const bool dev = is_dev(p.storage);
    a.fin = ws + (h->cur ? h->lay.fB : h->lay.fA);
    a.fout = ws + (h->cur ? h->lay.fA : h->lay.fB);
    a.rin = dev ? reinterpret_cast<const float*>(ws + (h->cur ? h->lay.rB : h->lay.rA)) : nullptr;
    a.rout = dev ? reinterpret_cast<float*>(ws + (h->cur ? h->lay.rA : h->lay.rB)) : nullptr;
    if (bufs) {
        a.fin = bufs->fin;
        a.fout = bufs->fout;
        a.rin = bufs->rin;
        a.rout = bufs->rout;
    }
    a.nbr = reinterpret_cast<const uint32_t*>(ws + h->lay.nbr);
    a.wet = reinterpret_cast<const R*>(ws + h->lay.wet);
    a.NA = h->NA;
    a.NB = h->NB;
    a.NC_ = h->NCc;
    a.N = h->N;
    a.common_u = p.common_velocity ? 1 : 0;
    a.wet_uniform = h->wet_uniform ? 1 : 0;
    a.has_zc = 0;
    const int q = q_of(p.lattice);
    for (int k = 0; k < p.n_comp; ++k) {
        a.psi_cs[k] = p.psi_kind[k] == LBM_PSI_CS;
        a.wet_drho[k] = p.wet_mode[k] == LBM_WET_DRHO;
        a.wet_val[k] = (R)p.wet[k];
        a.omega[k] = (R)(1.0 / p.tau[k]);
        for (int m = 0; m < q; ++m) {
            const double nrm = p.lattice == LBM_D2Q9 ? lbm::mrt_norm<lbm::LAT_D2Q9>(m) : lbm::mrt_norm<lbm::LAT_D3Q19>(m);
            a.srate[k][m] = (R)(p.mrt_s[k][m] / nrm);
        }
        a.eos_a[k] = (R)p.eos_a[k];
        a.eos_b[k] = (R)p.eos_b[k];
        a.eos_RT[k] = (R)(p.eos_R[k] * p.eos_T[k]);
        a.alpha[k] = (R)p.alpha[k];
        a.ginv[k] = p.g[k][k] != 0.0 ? (R)(1.0 / p.g[k][k]) : (R)0;
        a.A[k] = (R)p.A[k];
        if (p.A[k] != 0.0 && p.psi_kind[k] == LBM_PSI_CS) a.has_zc = 1;
        for (int kk = 0; kk < p.n_comp; ++kk) a.g[k][kk] = (R)p.g[k][kk];
        a.rho_min[k] = (R)p.rho_min[k];
        a.rho_max[k] = (R)p.rho_max[k];
        a.kq[k] = (R)(p.kappa[k] * p.g[k][k]);
        for (int r = 0; r < 2; ++r) {
            a.res_rho[r][k] = (R)p.res_rho[r][k];
            a.res_abb[r][k] = (R)h->res_active[r][k];
        }
    }
    for (int d = 0; d < 3; ++d) a.body[d] = (R)p.body_accel[d];
}
}  // namespace lbmi
