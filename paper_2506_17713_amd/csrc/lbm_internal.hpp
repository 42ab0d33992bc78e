// Internals of liblbm.so shared by the forward (lbm_api.hip) and adjoint
// (lbm_adjoint.hip) translation units: workspace layout and the handle.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdint>

#include "lbm.h"
#include "lbm_device.hpp"

namespace lbmi {

constexpr int kRedBlocks = 1024;  // partial sums of the first reduction pass
constexpr int kRedThreads = 256;
constexpr int kStatSlots = 16;    // doubles per partial / in the result

struct Layout {
    size_t fA, fB, rA, rB, nbr, wet, mrho, mu, uxprev, partial, dstats, conv_part, total;
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
};

namespace lbmi {
// One fused step from b.fin to b.fout (the handle's own buffers are untouched).
hipError_t run_step_buffers(lbm_handle* h, const Buffers& b);
// Pointer to the handle's current state buffer.
inline void* state_ptr(lbm_handle* h) { return h->ws + (h->cur ? h->lay.fB : h->lay.fA); }
}  // namespace lbmi
