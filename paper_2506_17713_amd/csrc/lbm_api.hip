// C-ABI of liblbm.so: handle management, workspace carving, kernel dispatch
// and the FP64 reductions behind lbm_stats.  Declarations: include/lbm.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "lbm_internal.hpp"

using namespace lbm;
using namespace lbmi;

// Build-time tile configuration of the 3-D 32-bit kernels: the tile is
// LBM_TILE_A x LBM_TILE_B nodes in (x, y) (LBM_TILE_B_BGK for the BGK steps
// that take taller tiles, see tile_b), and LBM_CARRY selects whether
// own-node populations are carried in registers from the pull to the
// collision.
#ifndef LBM_TILE_A
#define LBM_TILE_A 64
#endif
#ifndef LBM_TILE_B
#define LBM_TILE_B 4
#endif
#ifndef LBM_TILE_B_BGK
#define LBM_TILE_B_BGK 8
#endif
#ifndef LBM_CARRY
#define LBM_CARRY 1
#endif

namespace {


int validate(const lbm_params* p) {
    if (!p) return LBM_ERR_ARG;
    if (p->lattice != LBM_D2Q9 && p->lattice != LBM_D3Q19) return LBM_ERR_ARG;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return LBM_ERR_ARG;
    if (p->lattice == LBM_D2Q9 && p->nz != 1) return LBM_ERR_ARG;
    const long long N = (long long)p->nx * p->ny * p->nz;
    if (N >= (1LL << 31)) return LBM_ERR_ARG;
    // in-plane byte offsets are 32-bit (8-byte values at most)
    if ((long long)p->nx * (p->lattice == LBM_D2Q9 ? 1 : p->ny) >= (1LL << 29)) return LBM_ERR_ARG;
    if (p->n_comp < 1 || p->n_comp > 2) return LBM_ERR_ARG;
    if (p->collision != LBM_BGK && p->collision != LBM_MRT && p->collision != LBM_CLBM) return LBM_ERR_ARG;
    // central moments: one D2Q9 component (Eq. 3, Eq. 7-8)
    if (p->collision == LBM_CLBM && (p->lattice != LBM_D2Q9 || p->n_comp != 1)) return LBM_ERR_UNSUPPORTED;
    if (p->storage < LBM_STORE_F64 || p->storage > LBM_STORE_F32_F64) return LBM_ERR_ARG;
    if (p->check_every < 0) return LBM_ERR_ARG;
    for (int i = 0; i < 4; ++i)
        if (p->reserved[i] != 0) return LBM_ERR_ARG;
    if (p->reserved2 != 0) return LBM_ERR_ARG;
    if (p->layout != LBM_LAYOUT_DENSE && p->layout != LBM_LAYOUT_FLUID) return LBM_ERR_ARG;
    // fluid-only layout: D3Q19, BGK or MRT
    if (p->layout == LBM_LAYOUT_FLUID && (p->lattice != LBM_D3Q19 || p->collision == LBM_CLBM))
        return LBM_ERR_UNSUPPORTED;
    for (int k = 0; k < p->n_comp; ++k) {
        if (!(p->tau[k] > 0.5) || !std::isfinite(p->tau[k])) return LBM_ERR_ARG;
        if (p->psi_kind[k] != LBM_PSI_CS && p->psi_kind[k] != LBM_PSI_DENSITY) return LBM_ERR_ARG;
        if (p->wet_mode[k] != LBM_WET_PHI && p->wet_mode[k] != LBM_WET_DRHO) return LBM_ERR_ARG;
        if (!(p->rho_min[k] <= p->rho_max[k])) return LBM_ERR_ARG;
        if (!std::isfinite(p->kappa[k])) return LBM_ERR_ARG;
        // the surface-tension source is defined for D2Q9 MRT (Eq. 15)
        if (p->kappa[k] != 0.0 && (p->lattice != LBM_D2Q9 || p->collision != LBM_MRT)) return LBM_ERR_UNSUPPORTED;
        if (p->collision != LBM_BGK)
            for (int m = 0; m < q_of(p->lattice); ++m)
                if (!(p->mrt_s[k][m] >= 0.0 && p->mrt_s[k][m] < 2.0)) return LBM_ERR_ARG;
        if (p->psi_kind[k] == LBM_PSI_CS) {
            // Eq. 12 needs g_kk < 0; the square-root argument must stay
            // non-negative over the densities the limiter admits
            if (!(p->g[k][k] < 0.0)) return LBM_ERR_ARG;
            if (!(p->eos_b[k] > 0.0) || !(p->eos_T[k] > 0.0)) return LBM_ERR_ARG;
            const double hi = p->rho_max[k];
            if (hi < 1e10) {
                for (int s = 0; s <= 64; ++s) {
                    const double r = p->rho_min[k] + (hi - p->rho_min[k]) * s / 64.0;
                    const double eta = p->eos_b[k] * r / 4.0;
                    if (eta >= 1.0) return LBM_ERR_ARG;
                    const double pe = r * p->eos_R[k] * p->eos_T[k] * (1 + eta + eta * eta - eta * eta * eta) /
                                          ((1 - eta) * (1 - eta) * (1 - eta)) -
                                      p->eos_a[k] * r * r;
                    if (p->alpha[k] * pe - r / 3.0 > 1e-12) return LBM_ERR_ARG;
                }
            }
        }
    }
    return LBM_OK;
}

Layout layout_of(const lbm_params* p) {
    Layout L{};
    const size_t N = (size_t)p->nx * p->ny * p->nz;
    const size_t nc = p->n_comp, q = q_of(p->lattice);
    const size_t sb = store_bytes(p->storage), rb = real_bytes(p->storage);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    // lbm_init stages the mask, rho0 and u0 in the second buffer
    const size_t stage = align256(N) + align256(nc * N * rb) + align256(3 * N * rb);
    // the fluid layout's rows have a stride of N rounded up to 64
    const bool fl = p->layout == LBM_LAYOUT_FLUID;
    const size_t NT = fl ? (N + 63) / 64 * 64 : N;
    const size_t pop = nc * q * NT * sb;
    L.fA = take(pop);
    L.fB = take(pop > stage ? pop : stage);
    L.rA = take(is_dev(p->storage) ? nc * NT * 4 : 0);
    L.rB = take(is_dev(p->storage) ? nc * NT * 4 : 0);
    L.nbr = take(N * 4);
    L.wet = take(nc * N * rb);
    L.mrho = take(nc * N * rb);
    L.mu = take(3 * N * rb);
    L.uxprev = take(N * rb);
    L.partial = take((size_t)kRedBlocks * kStatSlots * 8);
    L.dstats = take(kStatSlots * 8 + 8);
    // convective outlet: partial sums of the mean outward velocity
    const size_t plane = (size_t)p->nx * (p->lattice == LBM_D2Q9 ? 1 : p->ny);
    L.conv_part = take(((plane + kConvThreads - 1) / kConvThreads) * 16);
    L.ftab = take(fl ? (q - 1) * NT * 4 : 0);
    L.frho = take(fl ? nc * NT * rb : 0);
    L.fpsi = take(fl ? nc * NT * rb : 0);
    L.fU = take(fl ? nc * NT * rb : 0);
    L.fdmap = take(fl ? NT * 4 : 0);
    L.femap = take(fl ? N * 4 : 0);
    L.total = off;
    return L;
}

}  // namespace

namespace {

// Tile height of a step kernel.  For BGK with one FP32 component or two
// 16-bit ones, 64 x 8 tiles at 2 waves per SIMD beat 64 x 4 at 3: a taller
// tile pulls fewer halo positions per node (4 % and 7 % faster).  MRT, two
// FP32 components and one 16-bit component need the third wave (10-25 %
// slower with 64 x 8).
template <int LAT, int NC, int ST, int COLL, bool MOM>
constexpr int tile_b() {
    if (LAT == LAT_D2Q9) return 1;
    if (ST == ST_F64 || ST == ST_F32D) return 4;
    constexpr bool dev = ST == ST_F16 || ST == ST_BF16;
    if (COLL == COLL_BGK && !MOM && ((NC == 1 && ST == ST_F32) || (NC == 2 && dev))) return LBM_TILE_B_BGK;
    return LBM_TILE_B;
}

// Own-node populations stay in registers between pull and collision where
// three sets fit (one component, 32-bit arithmetic).
template <int LAT, int NC, int ST>
constexpr bool CARRY_OF() {
    return LBM_CARRY && NC == 1 && ST != ST_F64 && ST != ST_F32D;
}

template <int LAT, int NC, int ST, int COLL, bool MOM>
hipError_t launch_step(lbm_handle* h, StepArgs<typename Store<ST>::R>& a) {
    constexpr int TA = LAT == LAT_D2Q9 ? 64 : LBM_TILE_A;
    constexpr int TB = tile_b<LAT, NC, ST, COLL, MOM>();
    a.tiles_a = (h->NA + TA - 1) / TA;
    a.tiles_b = (h->NB + TB - 1) / TB;
    const int tiles = a.tiles_a * a.tiles_b;
    int chunk = h->chunk_override;
    if (chunk <= 0) {
        // On a mostly fluid lattice, as many chunks as let every workgroup of
        // the launch be resident at once (one round): all tiles start
        // together and none waits for a second round.  256^3: 3 chunks of 86
        // planes, 3 % faster than 8 chunks of 32 (FP16 deviation storage 10 %).
        // Porous media are the exception: their tiles hold very different
        // amounts of fluid, and many short chunks (about 2048 workgroups)
        // balance the load better than one long round (400^3 two-component
        // pack: 8 % faster with FP32, 30 % with 16-bit storage).  At least
        // 16 planes per chunk in 3-D (4 in 2-D): a chunk pulls 4 planes beyond
        // its own (the rho ring), so short chunks of small lattices cost more
        // than the extra workgroups gain (128^3: 16 beats 8 by 10 %).
        static int slots = 0;  // resident workgroups of this kernel on the device
        if (slots == 0 && h->mostly_fluid) {
            int per_cu = 0, cus = 0, dev = 0;
            if (hipGetDevice(&dev) == hipSuccess &&
                hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
                hipOccupancyMaxActiveBlocksPerMultiprocessor(
                    &per_cu, reinterpret_cast<const void*>(&k_step<LAT, NC, ST, COLL, MOM, TA, TB, CARRY_OF<LAT, NC, ST>()>),
                    TA * TB, 0) == hipSuccess &&
                per_cu > 0 && cus > 0)
                slots = per_cu * cus;
            else
                slots = 2048;
        }
        int want = h->mostly_fluid ? slots / tiles : (2048 + tiles - 1) / tiles;
        if (want < 1) want = 1;
        chunk = (h->NCc + want - 1) / want;
        const int minc = LAT == LAT_D2Q9 ? 4 : 16;
        if (chunk < minc) chunk = minc;
    }
    // an outlet plane (the last one) must not open a chunk's ring: its
    // density is copied from the ring's plane below it
    if (h->conv_plane >= 0 && chunk < 2) chunk = 2;
    if (chunk > h->NCc) chunk = h->NCc;
    a.chunk = chunk;
    const int nchunks = (h->NCc + chunk - 1) / chunk;
    const int nblk = tiles * nchunks;
    constexpr bool CARRY = CARRY_OF<LAT, NC, ST>();
    hipLaunchKernelGGL((k_step<LAT, NC, ST, COLL, MOM, TA, TB, CARRY>), dim3(nblk), dim3(TA * TB), 0,
                       h->stream, a);
    return hipGetLastError();
}

template <int LAT, int NC, int ST>
hipError_t dispatch_coll(lbm_handle* h, bool mom, StepArgs<typename Store<ST>::R>& a) {
    if (mom) return launch_step<LAT, NC, ST, COLL_BGK, true>(h, a);
    if (h->p.collision == LBM_MRT) return launch_step<LAT, NC, ST, COLL_MRT, false>(h, a);
    if constexpr (LAT == LAT_D2Q9 && NC == 1)
        if (h->p.collision == LBM_CLBM) return launch_step<LAT, NC, ST, COLL_CLBM, false>(h, a);
    return launch_step<LAT, NC, ST, COLL_BGK, false>(h, a);
}

template <int LAT, int NC>
hipError_t dispatch_store(lbm_handle* h, bool mom, int comp, void* rho, void* u, const Buffers* bufs) {
    switch (h->p.storage) {
        case LBM_STORE_F64: {
            StepArgs<double> a;
            fill_args(h, a, bufs);
            a.mom_comp = comp;
            a.mom_rho = (double*)rho;
            a.mom_u = (double*)u;
            return dispatch_coll<LAT, NC, ST_F64>(h, mom, a);
        }
        case LBM_STORE_F32: {
            StepArgs<float> a;
            fill_args(h, a, bufs);
            a.mom_comp = comp;
            a.mom_rho = (float*)rho;
            a.mom_u = (float*)u;
            return dispatch_coll<LAT, NC, ST_F32>(h, mom, a);
        }
        case LBM_STORE_F32_F64: {
            StepArgs<double> a;
            fill_args(h, a, bufs);
            a.mom_comp = comp;
            a.mom_rho = (double*)rho;
            a.mom_u = (double*)u;
            return dispatch_coll<LAT, NC, ST_F32D>(h, mom, a);
        }
        case LBM_STORE_F16DEV: {
            StepArgs<float> a;
            fill_args(h, a, bufs);
            a.mom_comp = comp;
            a.mom_rho = (float*)rho;
            a.mom_u = (float*)u;
            return dispatch_coll<LAT, NC, ST_F16>(h, mom, a);
        }
        default: {
            StepArgs<float> a;
            fill_args(h, a, bufs);
            a.mom_comp = comp;
            a.mom_rho = (float*)rho;
            a.mom_u = (float*)u;
            return dispatch_coll<LAT, NC, ST_BF16>(h, mom, a);
        }
    }
}

// Convective outlet after a step, on the handle's buffers before the swap:
// the mean outward velocity of the plane below the outlet, then the
// populations that stream in from the outlet at the next pull.
template <int LAT, int NC, int ST>
hipError_t conv_launch(lbm_handle* h) {
    using R = typename Store<ST>::R;
    StepArgs<R> a;
    fill_args(h, a, nullptr);
    const int plane = h->NA * h->NB;
    const int nblk = (plane + kConvThreads - 1) / kConvThreads;
    const int co = h->conv_plane, ci = (co + h->NCc - 1) % h->NCc;
    double* part = reinterpret_cast<double*>(h->ws + h->lay.conv_part);
    hipLaunchKernelGGL((k_conv_u<LAT, NC, ST>), dim3(nblk), dim3(kConvThreads), 0, h->stream, a, ci, part);
    hipLaunchKernelGGL((k_conv_ghost<LAT, NC, ST>), dim3(nblk), dim3(kConvThreads), 0, h->stream, a, co,
                       (const double*)part, nblk);
    return hipGetLastError();
}

template <int LAT, int NC>
hipError_t conv_store(lbm_handle* h) {
    switch (h->p.storage) {
        case LBM_STORE_F64: return conv_launch<LAT, NC, ST_F64>(h);
        case LBM_STORE_F32: return conv_launch<LAT, NC, ST_F32>(h);
        case LBM_STORE_F32_F64: return conv_launch<LAT, NC, ST_F32D>(h);
        default: return hipErrorInvalidValue;  // rejected at lbm_init
    }
}

hipError_t run_conv(lbm_handle* h) {
    if (h->conv_plane < 0) return hipSuccess;
    if (h->p.layout == LBM_LAYOUT_FLUID) return fluid_conv(h);
    if (h->p.lattice == LBM_D2Q9)
        return h->p.n_comp == 1 ? conv_store<LAT_D2Q9, 1>(h) : conv_store<LAT_D2Q9, 2>(h);
    return h->p.n_comp == 1 ? conv_store<LAT_D3Q19, 1>(h) : conv_store<LAT_D3Q19, 2>(h);
}

hipError_t run_kernel(lbm_handle* h, bool mom, int comp = -1, void* rho = nullptr, void* u = nullptr,
                      const Buffers* bufs = nullptr) {
    if (h->p.layout == LBM_LAYOUT_FLUID) {
        if (bufs) return hipErrorInvalidValue;  // explicit buffers: the adjoint only, dense layout
        return mom ? fluid_moments(h, comp, rho, u) : fluid_step(h);
    }
    const bool d2 = h->p.lattice == LBM_D2Q9;
    if (d2) {
        if (h->p.n_comp == 1) return dispatch_store<LAT_D2Q9, 1>(h, mom, comp, rho, u, bufs);
        return dispatch_store<LAT_D2Q9, 2>(h, mom, comp, rho, u, bufs);
    }
    if (h->p.n_comp == 1) return dispatch_store<LAT_D3Q19, 1>(h, mom, comp, rho, u, bufs);
    return dispatch_store<LAT_D3Q19, 2>(h, mom, comp, rho, u, bufs);
}

// ---------------------------------------------------------------------------
// Reductions (FP64 accumulators, wavefront shuffles, fixed order).
// Slots: 0,1 mass; 2,3,4 momentum; 5 sum|ux-prev|; 6 sum|ux|; 7 sum ux;
//        8 non-wetting count; 9 fluid count; 10 non-finite; 11 negative;
//        in the window of planes: 12 / 13 pressure sums of the non-wetting /
//        wetting nodes, 14 / 15 their counts (Sec. 3.4.3).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

constexpr int kSlotsUsed = 16;

template <class R>
__global__ void __launch_bounds__(kRedThreads)
    k_reduce1(const R* __restrict__ rho, const R* __restrict__ u, R* __restrict__ uxprev,
              const uint32_t* __restrict__ nbr, double* __restrict__ partial, int N, int nc,
              int have_prev, R rho_mid, StepArgs<R> P, int plane, int w0, int w1) {
    double acc[kSlotsUsed];
#pragma unroll
    for (int s = 0; s < kSlotsUsed; ++s) acc[s] = 0.0;
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < N; n += gridDim.x * blockDim.x) {
        if (nbr[n] & 1u) continue;
        const double r0 = rho[n];
        const double r1 = nc > 1 ? (double)rho[(size_t)N + n] : 0.0;
        const double rt = r0 + r1;
        const double ux = u[n], uy = u[(size_t)N + n], uz = u[2 * (size_t)N + n];
        const double prev = have_prev ? (double)uxprev[n] : 0.0;
        uxprev[n] = (R)ux;
        acc[0] += r0;
        acc[1] += r1;
        acc[2] += rt * ux;
        acc[3] += rt * uy;
        acc[4] += rt * uz;
        acc[5] += fabs(ux - prev);
        acc[6] += fabs(ux);
        acc[7] += ux;
        const bool nw = nc > 1 ? r0 >= r1 : r0 < (double)rho_mid;
        acc[8] += nw ? 1.0 : 0.0;
        acc[9] += 1.0;
        const int c = n / plane;
        if (c >= w0 && c < w1) {
            // p = c_s^2 sum_k rho^k + (1/2) sum_kk' g_kk' psi^k psi^k'
            R ps0, ps1 = (R)0, U;
            psi_of(P, 0, (R)r0, ps0, U);
            if (nc > 1) psi_of(P, 1, (R)r1, ps1, U);
            const double s0 = ps0, s1 = ps1;
            double pr = rt / 3.0 + 0.5 * (double)P.g[0][0] * s0 * s0;
            if (nc > 1) pr += (double)P.g[0][1] * s0 * s1 + 0.5 * (double)P.g[1][1] * s1 * s1;
            acc[nw ? 12 : 13] += pr;
            acc[nw ? 14 : 15] += 1.0;
        }
        const bool fin = std::isfinite(r0) && std::isfinite(r1) && std::isfinite(ux) && std::isfinite(uy) &&
                         std::isfinite(uz);
        acc[10] += fin ? 0.0 : 1.0;
        acc[11] += (r0 < 0.0 || r1 < 0.0) ? 1.0 : 0.0;
    }
    __shared__ double sh[kRedThreads / 64][kSlotsUsed];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int s = 0; s < kSlotsUsed; ++s) {
        const double v = wave_sum(acc[s]);
        if (lane == 0) sh[wv][s] = v;
    }
    __syncthreads();
    if (threadIdx.x < kSlotsUsed) {
        double v = 0.0;
        for (int w = 0; w < kRedThreads / 64; ++w) v += sh[w][threadIdx.x];
        partial[(size_t)blockIdx.x * kStatSlots + threadIdx.x] = v;
    }
}

__global__ void k_reduce2(const double* __restrict__ partial, double* __restrict__ out, int nblk) {
    // one wavefront per slot, fixed order
    const int s = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (s >= kSlotsUsed) return;
    double v = 0.0;
    for (int b = lane; b < nblk; b += 64) v += partial[(size_t)b * kStatSlots + s];
    v = wave_sum(v);
    if (lane == 0) {
        out[s] = v;
        if (s == 10 || s == 11) {
            // sticky failure flag after the result slots
            if (v > 0.0) reinterpret_cast<unsigned long long*>(out + kStatSlots)[0] = 1ull;
        }
    }
}

hipError_t enqueue_stats(lbm_handle* h) {
    char* ws = h->ws;
    const size_t rb = real_bytes(h->p.storage);
    hipError_t e;
    for (int k = 0; k < h->p.n_comp; ++k) {
        e = run_kernel(h, true, k, ws + h->lay.mrho + (size_t)k * h->N * rb, nullptr);
        if (e != hipSuccess) return e;
    }
    e = run_kernel(h, true, -1, nullptr, ws + h->lay.mu);
    if (e != hipSuccess) return e;
    const double mid = 0.5 * (h->p.rho_min[0] + h->p.rho_max[0]);
    const uint32_t* nbr = reinterpret_cast<const uint32_t*>(ws + h->lay.nbr);
    double* part = reinterpret_cast<double*>(ws + h->lay.partial);
    const int plane = h->NA * h->NB;
    int w0 = h->p.window[0], w1 = h->p.window[1];
    if (w1 <= w0) {
        w0 = 0;
        w1 = h->NCc;
    }
    if (real_bytes(h->p.storage) == 8) {
        StepArgs<double> a;
        fill_args(h, a, nullptr);
        hipLaunchKernelGGL(k_reduce1<double>, dim3(kRedBlocks), dim3(kRedThreads), 0, h->stream,
                           reinterpret_cast<const double*>(ws + h->lay.mrho),
                           reinterpret_cast<const double*>(ws + h->lay.mu),
                           reinterpret_cast<double*>(ws + h->lay.uxprev), nbr, part, h->N, h->p.n_comp,
                           h->have_prev ? 1 : 0, mid, a, plane, w0, w1);
    } else {
        StepArgs<float> a;
        fill_args(h, a, nullptr);
        hipLaunchKernelGGL(k_reduce1<float>, dim3(kRedBlocks), dim3(kRedThreads), 0, h->stream,
                           reinterpret_cast<const float*>(ws + h->lay.mrho),
                           reinterpret_cast<const float*>(ws + h->lay.mu),
                           reinterpret_cast<float*>(ws + h->lay.uxprev), nbr, part, h->N, h->p.n_comp,
                           h->have_prev ? 1 : 0, (float)mid, a, plane, w0, w1);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce2, dim3(1), dim3(kSlotsUsed * 64), 0, h->stream, part,
                       reinterpret_cast<double*>(ws + h->lay.dstats), kRedBlocks);
    h->have_prev = true;
    return hipGetLastError();
}

template <class R>
std::vector<R> to_real(const double* src, size_t n) {
    std::vector<R> v(n);
    for (size_t i = 0; i < n; ++i) v[i] = (R)src[i];
    return v;
}

template <int LAT, int NC, int ST>
hipError_t launch_init(lbm_handle* h, const void* rho0, const void* u0) {
    const int N = h->N;
    const int blk = 256, grid = (N + blk - 1) / blk;
    using R = typename Store<ST>::R;
    ResRho res;
    for (int r = 0; r < 2; ++r)
        for (int k = 0; k < 2; ++k) res.r[r][k] = h->res_active[r][k];
    hipLaunchKernelGGL((k_init<LAT, NC, ST>), dim3(grid), dim3(blk), 0, h->stream, (const R*)rho0,
                       (const R*)u0, reinterpret_cast<const uint32_t*>(h->ws + h->lay.nbr), h->ws + h->lay.fA,
                       is_dev(h->p.storage) ? reinterpret_cast<float*>(h->ws + h->lay.rA) : nullptr, h->NA,
                       h->NB, h->NCc, res);
    return hipGetLastError();
}

template <int LAT, int NC>
hipError_t init_store(lbm_handle* h, const void* rho0, const void* u0) {
    switch (h->p.storage) {
        case LBM_STORE_F64: return launch_init<LAT, NC, ST_F64>(h, rho0, u0);
        case LBM_STORE_F32: return launch_init<LAT, NC, ST_F32>(h, rho0, u0);
        case LBM_STORE_F32_F64: return launch_init<LAT, NC, ST_F32D>(h, rho0, u0);
        case LBM_STORE_F16DEV: return launch_init<LAT, NC, ST_F16>(h, rho0, u0);
        default: return launch_init<LAT, NC, ST_BF16>(h, rho0, u0);
    }
}

}  // namespace

hipError_t lbmi::run_step_buffers(lbm_handle* h, const Buffers& b) { return run_kernel(h, false, -1, nullptr, nullptr, &b); }

extern "C" {

const char* lbm_strerror(int code) {
    switch (code) {
        case LBM_OK: return "ok";
        case LBM_ERR_ARG: return "invalid argument";
        case LBM_ERR_UNSUPPORTED: return "unsupported configuration";
        case LBM_ERR_HIP: return "HIP runtime error";
        case LBM_ERR_NONFINITE: return "non-finite or negative density detected";
        case LBM_ERR_SPACE: return "workspace too small";
        case LBM_ERR_OOM: return "out of host memory";
        default: return "unknown error";
    }
}

int lbm_workspace_size(const lbm_params* p, size_t* bytes_out) {
    int rc = validate(p);
    if (rc) return rc;
    if (!bytes_out) return LBM_ERR_ARG;
    *bytes_out = layout_of(p).total;
    return LBM_OK;
}

int lbm_init(const lbm_params* p, const uint8_t* mask, const double* rho0, const double* u0,
             const double* wet, void* workspace, size_t ws_bytes, void* stream, lbm_handle** out) {
    if (!out || !mask || !rho0 || !workspace) return LBM_ERR_ARG;
    *out = nullptr;
    int rc = validate(p);
    if (rc) return rc;
    Layout lay = layout_of(p);
    if (ws_bytes < lay.total) return LBM_ERR_SPACE;
    if (((uintptr_t)workspace & 255u) != 0) return LBM_ERR_ARG;
    const size_t N = (size_t)p->nx * p->ny * p->nz;
    const int nc = p->n_comp;
    // open boundaries: reservoir nodes fill whole planes of the marching axis,
    // one reservoir per plane, with positive densities, and no fluid plane
    // lies between two reservoir planes
    const size_t plane = (size_t)p->nx * (p->lattice == LBM_D2Q9 ? 1 : p->ny);
    const size_t n_planes = N / plane;
    std::vector<int> kind(n_planes, 0);  // 0 none, 1 fluid, 2 / 3 reservoir, 4 outlet
    bool has_res = false;
    int conv_plane = -1;
    for (size_t c = 0; c < n_planes; ++c) {
        const uint8_t* m = mask + c * plane;
        const uint8_t m0 = m[0];
        size_t nres = 0, nfl = 0;
        for (size_t i = 0; i < plane; ++i) {
            if (m[i] > 4) return LBM_ERR_ARG;
            if (m[i] >= 2) {
                if (m[i] != m0) return LBM_ERR_ARG;
                ++nres;
            }
            if (m[i] == 0) ++nfl;
        }
        if (nres && nres != plane) return LBM_ERR_ARG;
        kind[c] = nres ? m0 : (nfl ? 1 : 0);
        if (nres) {
            has_res = true;
            const int r = m0 == 4 ? 1 : m0 - 2;  // the outlet's fallback density is reservoir 1's
            for (int k = 0; k < nc; ++k)
                if (!std::isfinite(p->res_rho[r][k]) || !(p->res_rho[r][k] > 0.0)) return LBM_ERR_ARG;
        }
        if (m0 == 4 && nres) {
            if (conv_plane >= 0) return LBM_ERR_ARG;  // one outlet plane
            conv_plane = (int)c;
        }
    }
    for (size_t c = 0; c < n_planes && has_res; ++c)
        if (kind[c] == 1 && kind[(c + n_planes - 1) % n_planes] >= 2 && kind[(c + 1) % n_planes] >= 2)
            return LBM_ERR_ARG;
    if (conv_plane >= 0) {
        // the last plane of the marching axis, fluid below it and none in
        // the first plane (above it across the wrap); full-precision storage
        if (n_planes < 4 || conv_plane != (int)n_planes - 1 || kind[n_planes - 2] != 1 || kind[0] == 1)
            return LBM_ERR_ARG;
        if (is_dev(p->storage)) return LBM_ERR_UNSUPPORTED;
    }
    size_t n_solid = 0;
    for (size_t n = 0; n < N; ++n) {
        if (mask[n]) {
            ++n_solid;
            continue;
        }
        for (int k = 0; k < nc; ++k) {
            const double r = rho0[k * N + n];
            if (!std::isfinite(r) || r <= 0.0) return LBM_ERR_ARG;
        }
        if (u0)
            for (int d = 0; d < 3; ++d)
                if (!std::isfinite(u0[d * N + n])) return LBM_ERR_ARG;
    }
    lbm_handle* h = new (std::nothrow) lbm_handle();
    if (!h) return LBM_ERR_OOM;
    h->p = *p;
    h->lay = lay;
    h->stream = (hipStream_t)stream;
    h->ws = (char*)workspace;
    h->N = (int)N;
    h->NA = p->nx;
    h->NB = p->lattice == LBM_D2Q9 ? 1 : p->ny;
    h->NCc = p->lattice == LBM_D2Q9 ? p->ny : p->nz;
    h->cur = 0;
    h->step = 0;
    h->since_check = 0;
    h->have_prev = false;
    h->wet_uniform = wet == nullptr;
    h->has_res = has_res;
    h->conv_plane = conv_plane;
    h->n_col = h->n_fl = h->n_sol = h->n_r1 = h->n_ext = h->fl_T = h->conv_lo = h->conv_hi = 0;
    std::memcpy(h->res_active, p->res_rho, sizeof(h->res_active));
    h->mostly_fluid = n_solid * 10 < N;
    // LBM_CHUNK (environment, tuning only): planes per workgroup along the
    // marching axis; unset or 0 chooses about 2048 workgroups per launch.
    const char* ch = std::getenv("LBM_CHUNK");
    h->chunk_override = ch ? std::atoi(ch) : 0;

    const size_t rb = real_bytes(p->storage);
    // stage mask, rho0 and u0 in the second population buffer
    char* stage = h->ws + lay.fB;
    char* d_mask = stage;
    char* d_rho = stage + align256(N);
    char* d_u = d_rho + align256(nc * N * rb);
    hipError_t e = hipSuccess;
    std::vector<double> hd;
    std::vector<float> hf;
    auto upload = [&](void* dst, const double* src, size_t n) -> hipError_t {
        if (rb == 8) return hipMemcpyAsync(dst, src, n * 8, hipMemcpyHostToDevice, h->stream);
        hf = to_real<float>(src, n);
        hipError_t r = hipMemcpyAsync(dst, hf.data(), n * 4, hipMemcpyHostToDevice, h->stream);
        if (r == hipSuccess) r = hipStreamSynchronize(h->stream);
        return r;
    };
    e = hipMemcpyAsync(d_mask, mask, N, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = upload(d_rho, rho0, nc * N);
    if (e == hipSuccess && u0) e = upload(d_u, u0, 3 * N);
    // wetting field
    if (e == hipSuccess) {
        if (wet) {
            e = upload(h->ws + lay.wet, wet, nc * N);
        } else {
            std::vector<double> uni(nc * N);
            for (int k = 0; k < nc; ++k)
                for (size_t n = 0; n < N; ++n) uni[k * N + n] = p->wet[k];
            e = upload(h->ws + lay.wet, uni.data(), nc * N);
            if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        }
    }
    if (e == hipSuccess) e = hipMemsetAsync(h->ws + lay.dstats, 0, kStatSlots * 8 + 8, h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(h->ws + lay.fA, 0, lay.fB - lay.fA, h->stream);
    if (e == hipSuccess) {
        const int blk = 256, grid = (int)((N + blk - 1) / blk);
        if (p->lattice == LBM_D2Q9)
            hipLaunchKernelGGL(k_nbr_words<LAT_D2Q9>, dim3(grid), dim3(blk), 0, h->stream,
                               (const uint8_t*)d_mask, (uint32_t*)(h->ws + lay.nbr), h->NA, h->NB, h->NCc);
        else
            hipLaunchKernelGGL(k_nbr_words<LAT_D3Q19>, dim3(grid), dim3(blk), 0, h->stream,
                               (const uint8_t*)d_mask, (uint32_t*)(h->ws + lay.nbr), h->NA, h->NB, h->NCc);
        e = hipGetLastError();
    }
    if (e == hipSuccess && p->layout == LBM_LAYOUT_FLUID) {
        rc = fluid_build(h);
        if (rc != LBM_OK) {
            delete h;
            return rc;
        }
        e = fluid_init(h, d_rho, u0 ? d_u : nullptr);
    } else if (e == hipSuccess) {
        const void* du = u0 ? d_u : nullptr;
        if (p->lattice == LBM_D2Q9)
            e = nc == 1 ? init_store<LAT_D2Q9, 1>(h, d_rho, du) : init_store<LAT_D2Q9, 2>(h, d_rho, du);
        else
            e = nc == 1 ? init_store<LAT_D3Q19, 1>(h, d_rho, du) : init_store<LAT_D3Q19, 2>(h, d_rho, du);
    }
    if (e == hipSuccess) e = hipMemsetAsync(h->ws + lay.fB, 0, lay.rA - lay.fB, h->stream);
    if (e == hipSuccess && lay.nbr > lay.rB) e = hipMemsetAsync(h->ws + lay.rB, 0, lay.nbr - lay.rB, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        delete h;
        return LBM_ERR_HIP;
    }
    *out = h;
    return LBM_OK;
}

int lbm_step(lbm_handle* h, int64_t nsteps) {
    if (!h || nsteps < 0) return LBM_ERR_ARG;
    for (int64_t s = 0; s < nsteps; ++s) {
        if (run_kernel(h, false) != hipSuccess) return LBM_ERR_HIP;
        if (run_conv(h) != hipSuccess) return LBM_ERR_HIP;
        std::memcpy(h->res_active, h->p.res_rho, sizeof(h->res_active));
        h->cur ^= 1;
        h->step += 1;
        if (h->p.check_every > 0 && ++h->since_check >= h->p.check_every) {
            h->since_check = 0;
            if (enqueue_stats(h) != hipSuccess) return LBM_ERR_HIP;
        }
    }
    return LBM_OK;
}

int lbm_moments(lbm_handle* h, int comp, void* rho_dev, void* u_dev) {
    if (!h || comp < -1 || comp >= h->p.n_comp) return LBM_ERR_ARG;
    if (!rho_dev && !u_dev) return LBM_OK;
    return run_kernel(h, true, comp, rho_dev, u_dev) == hipSuccess ? LBM_OK : LBM_ERR_HIP;
}

static int read_flag(lbm_handle* h, double* res) {
    double buf[kStatSlots + 1];
    if (hipMemcpyAsync(buf, h->ws + h->lay.dstats, sizeof(buf), hipMemcpyDeviceToHost, h->stream) != hipSuccess)
        return LBM_ERR_HIP;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return LBM_ERR_HIP;
    if (res) std::memcpy(res, buf, sizeof(double) * kStatSlots);
    unsigned long long flag;
    std::memcpy(&flag, &buf[kStatSlots], 8);
    if (flag) {
        hipMemsetAsync(h->ws + h->lay.dstats + kStatSlots * 8, 0, 8, h->stream);
        hipStreamSynchronize(h->stream);
        return LBM_ERR_NONFINITE;
    }
    return LBM_OK;
}

int lbm_stats(lbm_handle* h, lbm_stats_t* out) {
    if (!h || !out) return LBM_ERR_ARG;
    if (enqueue_stats(h) != hipSuccess) return LBM_ERR_HIP;
    double r[kStatSlots];
    const int rc = read_flag(h, r);
    if (rc == LBM_ERR_HIP) return rc;
    std::memset(out, 0, sizeof(*out));
    out->step = h->step;
    out->mass[0] = r[0];
    out->mass[1] = r[1];
    out->momentum[0] = r[2];
    out->momentum[1] = r[3];
    out->momentum[2] = r[4];
    out->residual = r[6] > 0.0 ? r[5] / r[6] : 0.0;
    out->saturation = r[9] > 0.0 ? r[8] / r[9] : 0.0;
    out->mean_ux = r[9] > 0.0 ? r[7] / r[9] : 0.0;
    out->n_fluid = (int64_t)r[9];
    out->nonfinite = (int32_t)r[10];
    out->negative = (int32_t)r[11];
    out->p_nonwetting = r[14] > 0.0 ? r[12] / r[14] : 0.0;
    out->p_wetting = r[15] > 0.0 ? r[13] / r[15] : 0.0;
    out->capillary_pressure = out->p_nonwetting - out->p_wetting;
    out->s_wetting = r[14] + r[15] > 0.0 ? r[15] / (r[14] + r[15]) : 0.0;
    return rc;
}

int lbm_sync(lbm_handle* h) {
    if (!h) return LBM_ERR_ARG;
    return read_flag(h, nullptr);
}

int lbm_set_reservoir(lbm_handle* h, int r, const double* rho) {
    if (!h || !rho || r < 0 || r > 1) return LBM_ERR_ARG;
    for (int k = 0; k < h->p.n_comp; ++k)
        if (!std::isfinite(rho[k]) || !(rho[k] > 0.0)) return LBM_ERR_ARG;
    // the populations of the next step stream in at this density; the pulls
    // take it up after that step (res_active)
    for (int k = 0; k < h->p.n_comp; ++k) h->p.res_rho[r][k] = rho[k];
    return LBM_OK;
}

// Nodes per population row of the state: the lattice, or the fluid-layout stride.
static size_t state_rows(const lbm_handle* h) {
    return h->p.layout == LBM_LAYOUT_FLUID ? (size_t)h->fl_T : (size_t)h->N;
}

int lbm_state_bytes(const lbm_handle* h, size_t* bytes_out) {
    if (!h || !bytes_out) return LBM_ERR_ARG;
    const size_t N = state_rows(h);
    *bytes_out = (size_t)h->p.n_comp * q_of(h->p.lattice) * N * store_bytes(h->p.storage) +
                 (is_dev(h->p.storage) ? (size_t)h->p.n_comp * N * 4 : 0);
    return LBM_OK;
}

int lbm_get_state(lbm_handle* h, void* dev_dst) {
    if (!h || !dev_dst) return LBM_ERR_ARG;
    const size_t N = state_rows(h);
    const size_t fb = (size_t)h->p.n_comp * q_of(h->p.lattice) * N * store_bytes(h->p.storage);
    hipError_t e = hipMemcpyAsync(dev_dst, h->ws + (h->cur ? h->lay.fB : h->lay.fA), fb,
                                  hipMemcpyDeviceToDevice, h->stream);
    if (e == hipSuccess && is_dev(h->p.storage))
        e = hipMemcpyAsync((char*)dev_dst + fb, h->ws + (h->cur ? h->lay.rB : h->lay.rA),
                           (size_t)h->p.n_comp * N * 4, hipMemcpyDeviceToDevice, h->stream);
    return e == hipSuccess ? LBM_OK : LBM_ERR_HIP;
}

int lbm_set_state(lbm_handle* h, const void* dev_src) {
    if (!h || !dev_src) return LBM_ERR_ARG;
    const size_t N = state_rows(h);
    const size_t fb = (size_t)h->p.n_comp * q_of(h->p.lattice) * N * store_bytes(h->p.storage);
    hipError_t e = hipMemcpyAsync(h->ws + (h->cur ? h->lay.fB : h->lay.fA), dev_src, fb,
                                  hipMemcpyDeviceToDevice, h->stream);
    if (e == hipSuccess && is_dev(h->p.storage))
        e = hipMemcpyAsync(h->ws + (h->cur ? h->lay.rB : h->lay.rA), (const char*)dev_src + fb,
                           (size_t)h->p.n_comp * N * 4, hipMemcpyDeviceToDevice, h->stream);
    return e == hipSuccess ? LBM_OK : LBM_ERR_HIP;
}

int lbm_reset(lbm_handle* h, const void* rho0_dev, const void* u0_dev) {
    if (!h || !rho0_dev) return LBM_ERR_ARG;
    h->cur = 0;
    h->step = 0;
    h->since_check = 0;
    h->have_prev = false;
    std::memcpy(h->res_active, h->p.res_rho, sizeof(h->res_active));
    const Layout& lay = h->lay;
    hipError_t e = hipMemsetAsync(h->ws + lay.dstats, 0, kStatSlots * 8 + 8, h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(h->ws + lay.fA, 0, lay.fB - lay.fA, h->stream);
    if (e == hipSuccess && h->p.layout == LBM_LAYOUT_FLUID) {
        e = fluid_init(h, rho0_dev, u0_dev);
    } else if (e == hipSuccess) {
        const int nc = h->p.n_comp;
        if (h->p.lattice == LBM_D2Q9)
            e = nc == 1 ? init_store<LAT_D2Q9, 1>(h, rho0_dev, u0_dev) : init_store<LAT_D2Q9, 2>(h, rho0_dev, u0_dev);
        else
            e = nc == 1 ? init_store<LAT_D3Q19, 1>(h, rho0_dev, u0_dev)
                        : init_store<LAT_D3Q19, 2>(h, rho0_dev, u0_dev);
    }
    if (e == hipSuccess) e = hipMemsetAsync(h->ws + lay.fB, 0, lay.rA - lay.fB, h->stream);
    if (e == hipSuccess && lay.nbr > lay.rB) e = hipMemsetAsync(h->ws + lay.rB, 0, lay.nbr - lay.rB, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    return e == hipSuccess ? LBM_OK : LBM_ERR_HIP;
}

void lbm_free(lbm_handle* h) { delete h; }

}  // extern "C"
