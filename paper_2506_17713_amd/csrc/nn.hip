// Kernels of the 3-D convolutional surrogate (include/lbm_nn.h).
//
// Convolution as an implicit GEMM on the MFMA matrix cores:
//   Y[co][p] = sum_k A[co][k] B[k][p],  k = (tap, ci),  B[k][p] = X[ci][p + off(tap)]
// BF16: a wave owns a 32 (co) x NT*32 (positions) tile and walks K in steps of
// 16 (v_mfma_f32_32x32x16_bf16, gfx950), each weight operand serving NT
// position tiles.  FP32: a wave owns a 32 x 32 tile and walks K in steps of 2
// (v_mfma_f32_32x32x2_f32).  Operand lane layout: lane l holds
// A[l % 32][k0 + l / 32 * kw + j] and B[k0 + l / 32 * kw + j][l % 32] (kw = 8
// for bf16, 1 for f32), and the accumulator element v of lane l is
// D[8 (v / 4) + 4 (l / 32) + v % 4][l % 32].
// Weight gradients are the GEMM dW[co][(ci,tap)] = sum_p dY[co][p] X[ci][p+off]
// with positions as the reduction dimension, split into chunks whose partial
// tiles are summed in a fixed order (deterministic).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "lbm.h"
#include "lbm_nn.h"

#ifndef LBM_NN_CONV_NT
#define LBM_NN_CONV_NT 2  // position tiles per wave of the BF16 convolution
#endif
#ifndef LBM_NN_CONV_LDS
#define LBM_NN_CONV_LDS 1  // BF16 convolution with the input brick staged in LDS (W >= 32)
#endif
#ifndef LBM_NN_CONV_16ROW
#define LBM_NN_CONV_16ROW 1  // 16-row MFMA tiles for layers of at most 16 output channels
#endif
// Brick of that kernel: 64 x BRICK_Y x BRICK_Z positions, BRICK_WAVES waves.
// 64 x 2 x 2 with 4 waves is the fastest measured: 64 x 4 x 2 (4 waves, two
// rows each) and 64 x 4 x 4 (8 waves) ran 13 % slower despite their smaller
// halo (fewer resident workgroups, more registers per wave).
#ifndef LBM_NN_BRICK_Y
#define LBM_NN_BRICK_Y 2
#endif
#ifndef LBM_NN_BRICK_Z
#define LBM_NN_BRICK_Z 2
#endif
#ifndef LBM_NN_BRICK_WAVES
#define LBM_NN_BRICK_WAVES 4
#endif

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short f2bf(float v) {
    uint32_t u = __float_as_uint(v);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (short)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

__host__ __device__ inline int cin_pad_of(int cin, int prec) { return prec == LBM_NN_BF16 ? (cin + 15) / 16 * 16 : (cin + 1) / 2 * 2; }
__host__ __device__ inline int cout_pad_of(int cout) { return (cout + 31) / 32 * 32; }

__device__ __forceinline__ int wrapc(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Four consecutive output channels co .. co + 3 of position p into the BF16
// channels-innermost copy yb[p][cop16] that the next convolution reads
// (channels at or beyond cout written as zero).
__device__ __forceinline__ void store_yb4(short* __restrict__ yb, int cop16, int p, int co, int cout, const float (&r)[4]) {
    if (co >= cop16) return;
    bf16x4 v;
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = co + j < cout ? f2bf(r[j]) : (short)0;
    *reinterpret_cast<bf16x4*>(yb + (size_t)p * cop16 + co) = v;
}

// packed layout: bf16  [tap][cin_pad/8][cout_pad][8] (four 32-bit words per entry)
//                fp32  [tap][cin_pad][cout_pad]
__global__ void k_pack(const float* __restrict__ W, int cout, int cin, int transpose, int prec,
                       uint32_t* __restrict__ out) {
    // logical layer after an optional transpose: (co', ci') = (ci, co), tap mirrored
    const int lo = transpose ? cin : cout, li = transpose ? cout : cin;
    const int cip = cin_pad_of(li, prec), cop = cout_pad_of(lo);
    const int total = 27 * cip * cop;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int co = idx % cop;
    const int ci = (idx / cop) % cip;
    const int tap = idx / (cop * cip);
    float v = 0.0f;
    if (co < lo && ci < li) {
        v = transpose ? W[((size_t)ci * cin + co) * 27 + (26 - tap)] : W[((size_t)co * cin + ci) * 27 + tap];
    }
    if (prec == LBM_NN_BF16) {
        const int cg = ci / 8, j = ci % 8;
        short* o = reinterpret_cast<short*>(out);
        o[(((size_t)tap * (cip / 8) + cg) * cop + co) * 8 + j] = f2bf(v);
    } else {
        reinterpret_cast<float*>(out)[((size_t)tap * cip + ci) * cop + co] = v;
    }
}

// Input of a BF16 convolution converted once: Xb[p][cin_pad] (BF16, channels
// innermost, zero beyond cin), so that a lane's B operand (8 channels at one
// position) is one 16-byte load.  A block transposes 64 positions through LDS:
// it reads each channel plane's 64 positions as one 256-byte row and writes
// the block's 64 x cin_pad values as one contiguous run of 16-byte words.
constexpr int kPackPos = 64, kPackMaxC = 128;

__global__ void __launch_bounds__(256) k_act_pack(const float* __restrict__ X, int cin, int cip, int64_t P,
                                                  s16x8* __restrict__ Xb) {
    __shared__ short sh[kPackMaxC][kPackPos + 2];  // [channel][position] (+2: fewer bank conflicts)
    const int64_t p0 = (int64_t)blockIdx.x * kPackPos;
    const int t = threadIdx.x, lp = t % kPackPos;
    const bool ok = p0 + lp < P;
    const int G = cip / 8;
    for (int cb = 0; cb < cip; cb += kPackMaxC) {  // channel chunks of at most 128
        const int nc = cip - cb < kPackMaxC ? cip - cb : kPackMaxC;
        if (cb > 0) __syncthreads();
        for (int cl = t / kPackPos; cl < nc; cl += 256 / kPackPos) {
            const int ci = cb + cl;
            sh[cl][lp] = (ci < cin && ok) ? f2bf(X[(size_t)ci * P + p0 + lp]) : (short)0;
        }
        __syncthreads();
        const int Gc = nc / 8;
        for (int w = t; w < kPackPos * Gc; w += 256) {
            const int pos = w / Gc, g = w % Gc;
            if (p0 + pos >= P) continue;
            s16x8 v;
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = sh[8 * g + j][pos];
            Xb[(size_t)(p0 + pos) * G + cb / 8 + g] = v;
        }
    }
}

// Epilogue of a 32-row tile at position p: bias, activation, skip; the FP32
// output Y[co][p] and / or the BF16 channels-innermost copy (either may be NULL).
__device__ __forceinline__ void epilogue32(const f32x16& acc, int p, int P, int co0, int kq, int cout,
                                           const float* __restrict__ bias, const float* __restrict__ skip, int relu,
                                           float* __restrict__ Y, short* __restrict__ yb) {
    const int cop16 = (cout + 15) / 16 * 16;
#pragma unroll
    for (int vg = 0; vg < 4; ++vg) {
        float r[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int co = co0 + 8 * vg + 4 * kq + j;
            r[j] = 0.0f;
            if (co < cout) {
                float t = acc[4 * vg + j] + (bias ? bias[co] : 0.0f);
                if (relu) t = t > 0.0f ? t : 0.0f;
                if (skip) t += skip[(size_t)co * P + p];
                r[j] = t;
                if (Y) Y[(size_t)co * P + p] = t;
            }
        }
        if (yb) store_yb4(yb, cop16, p, co0 + 8 * vg + 4 * kq, cout, r);
    }
}

// FP32 convolution: one wave per 32 (co) x 32 (positions) tile.
__global__ void __launch_bounds__(256)
    k_conv_f32(const float* __restrict__ X, int cin, const uint32_t* __restrict__ packed,
               const float* __restrict__ bias, const float* __restrict__ skip, float* __restrict__ Y, int cout, int D,
               int H, int W, int relu) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int P = D * H * W;
    const int p = (blockIdx.x * 4 + wave) * 32 + (lane & 31);
    const bool pok = p < P;
    const int pp = pok ? p : 0;
    const int x = pp % W, y = (pp / W) % H, z = pp / (W * H);
    const int co0 = blockIdx.y * 32;
    const int kq = lane >> 5;
    const int cip = cin_pad_of(cin, LBM_NN_FP32), cop = cout_pad_of(cout);
    f32x16 acc;
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
    const float* wp = reinterpret_cast<const float*>(packed);
    for (int tap = 0; tap < 27; ++tap) {
        const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
        const int q = (wrapc(z + dz, D) * H + wrapc(y + dy, H)) * W + wrapc(x + dx, W);
        for (int c2 = 0; c2 < cip; c2 += 2) {
            const int ci = c2 + kq;
            const float a = wp[((size_t)tap * cip + ci) * cop + co0 + (lane & 31)];
            const float b = (pok && ci < cin) ? X[(size_t)ci * P + q] : 0.0f;
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
        }
    }
    if (!pok) return;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int co = co0 + 8 * (v / 4) + 4 * kq + (v % 4);
        if (co < cout) {
            float r = acc[v] + (bias ? bias[co] : 0.0f);
            if (relu) r = r > 0.0f ? r : 0.0f;
            if (skip) r += skip[(size_t)co * P + p];
            Y[(size_t)co * P + p] = r;
        }
    }
}

// BF16 convolution: one wave per 32 (co) x NT*32 (positions) tile, K in steps
// of 16 channels of one tap.  The weight operand (8 channels of one output
// channel: 16 bytes) is loaded once for NT MFMAs; each input operand (8
// channels at one tap position of the channels-innermost copy Xb: 16 bytes) is
// one load.  The next step's operands are loaded before this step's MFMAs.
template <int NT>
__global__ void __launch_bounds__(256)
    k_conv_bf16(const short* __restrict__ Xb, int cin, const uint32_t* __restrict__ packed,
                const float* __restrict__ bias, const float* __restrict__ skip, float* __restrict__ Y,
                short* __restrict__ yb, int cout, int D, int H, int W, int relu) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int P = D * H * W;
    const int cip = cin_pad_of(cin, LBM_NN_BF16), cop = cout_pad_of(cout);
    const int co0 = blockIdx.y * 32;
    const int kq = lane >> 5;
    const int pbase = (blockIdx.x * 4 + wave) * (32 * NT) + (lane & 31);
    int px[NT], py[NT], pz[NT];
    bool pok[NT];
#pragma unroll
    for (int s = 0; s < NT; ++s) {
        const int p = pbase + 32 * s;
        pok[s] = p < P;
        const int pp = pok[s] ? p : 0;
        px[s] = pp % W;
        py[s] = (pp / W) % H;
        pz[s] = pp / (W * H);
    }
    f32x16 acc[NT];
#pragma unroll
    for (int s = 0; s < NT; ++s)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[s][v] = 0.0f;
    const s16x8* wp = reinterpret_cast<const s16x8*>(packed);
    const s16x8 zero = {0, 0, 0, 0, 0, 0, 0, 0};
    const int nc = cip / 16;        // K steps per tap
    const int nk = 27 * nc;         // K steps in all
    // operand addresses of K step t: tap = t / nc, channel block c = t % nc
    int q[NT];
    auto offsets = [&](int tap) {
        const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
#pragma unroll
        for (int s = 0; s < NT; ++s)
            q[s] = (wrapc(pz[s] + dz, D) * H + wrapc(py[s] + dy, H)) * W + wrapc(px[s] + dx, W);
    };
    auto load = [&](int t, s16x8& a, s16x8 (&b)[NT]) {
        const int tap = t / nc, c = t - tap * nc;
        a = wp[((size_t)tap * (cip / 8) + 2 * c + kq) * cop + co0 + (lane & 31)];
#pragma unroll
        for (int s = 0; s < NT; ++s)
            b[s] = pok[s] ? *reinterpret_cast<const s16x8*>(Xb + (size_t)q[s] * cip + 16 * c + 8 * kq) : zero;
    };
    s16x8 a0, b0[NT];
    offsets(0);
    load(0, a0, b0);
    for (int t = 0; t < nk; ++t) {
        s16x8 a1, b1[NT];
        if (t + 1 < nk) {
            if ((t + 1) % nc == 0) offsets((t + 1) / nc);
            load(t + 1, a1, b1);
        }
#pragma unroll
        for (int s = 0; s < NT; ++s)
            acc[s] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a0),
                                                             __builtin_bit_cast(bf16x8, b0[s]), acc[s], 0, 0, 0);
        a0 = a1;
#pragma unroll
        for (int s = 0; s < NT; ++s) b0[s] = b1[s];
    }
#pragma unroll
    for (int s = 0; s < NT; ++s) {
        if (!pok[s]) continue;
        const int p = pbase + 32 * s;
        epilogue32(acc[s], p, P, co0, kq, cout, bias, skip, relu, Y, yb);
    }
}

// BF16 convolution with the input staged in LDS: a workgroup of NW waves
// computes a brick of 64 (x) x BY (y) x BZ (z) positions for 32 output
// channels (BY * BZ / NW rows of 64 positions per wave, two 32-position MFMA
// tiles per row).  For each block of 16 input channels it stages the brick with
// its one-position halo (66 x (BY + 2) x (BZ + 2) positions x 32 bytes,
// periodic wrap) in LDS, then every tap takes its input operand there: the 27
// taps share one global read of each input.
constexpr int kBX = 64, kHX = kBX + 2;

template <int BY, int BZ>
constexpr int halo_positions() { return kHX * (BY + 2) * (BZ + 2); }

template <int BY, int BZ, int NW>
__global__ void __launch_bounds__(64 * NW)
    k_conv_bf16_lds(const short* __restrict__ Xb, int cin, const uint32_t* __restrict__ packed,
                    const float* __restrict__ bias, const float* __restrict__ skip, float* __restrict__ Y,
                    short* __restrict__ yb, int cout, int D, int H, int W, int relu) {
    constexpr int HY = BY + 2, HZ = BZ + 2, HALO = halo_positions<BY, BZ>();
    constexpr int RW = BY * BZ / NW;  // rows per wave
    static_assert(RW * NW == BY * BZ, "rows divide among the waves");
    __shared__ __align__(16) s16x8 sx[HALO * 2];  // [position][two halves of 8 channels]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int P = D * H * W;
    const int cip = cin_pad_of(cin, LBM_NN_BF16), cop = cout_pad_of(cout);
    const int nbx = (W + kBX - 1) / kBX, nby = (H + BY - 1) / BY;
    const int bx = blockIdx.x % nbx, by = (blockIdx.x / nbx) % nby, bz = blockIdx.x / (nbx * nby);
    const int x0 = bx * kBX, y0 = by * BY, z0 = bz * BZ;
    const int co0 = blockIdx.y * 32;
    const int kq = lane >> 5;
    int ly[RW], lz[RW];
    bool pok[RW][2];
#pragma unroll
    for (int r = 0; r < RW; ++r) {
        const int row = wave + NW * r;
        ly[r] = row % BY;
        lz[r] = row / BY;
#pragma unroll
        for (int s = 0; s < 2; ++s)
            pok[r][s] = x0 + 32 * s + (lane & 31) < W && y0 + ly[r] < H && z0 + lz[r] < D;
    }
    f32x16 acc[RW][2];
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[r][s][v] = 0.0f;
    const s16x8* wp = reinterpret_cast<const s16x8*>(packed);
    const s16x8* xg = reinterpret_cast<const s16x8*>(Xb);  // [position][cip / 8]
    const int g8 = cip / 8;
    for (int c = 0; c < cip / 16; ++c) {
        __syncthreads();  // the previous block's reads are done
        for (int i = threadIdx.x; i < HALO * 2; i += 64 * NW) {
            const int hp = i >> 1, half = i & 1;
            const int hx = hp % kHX, hy = (hp / kHX) % HY, hz = hp / (kHX * HY);
            int gx = wrapc(x0 + hx - 1, W), gy = wrapc(y0 + hy - 1, H), gz = wrapc(z0 + hz - 1, D);
            gx = gx < W ? gx : gx % W;  // bricks wider or taller than the lattice
            gy = gy < H ? gy : gy % H;
            gz = gz < D ? gz : gz % D;
            sx[i] = xg[((size_t)(gz * H + gy) * W + gx) * g8 + 2 * c + half];
        }
        __syncthreads();
        // the weights stay in global memory (cache hits): staged in LDS as
        // well they cost a workgroup per CU and ran 15 % slower
        s16x8 a0 = wp[((size_t)0 * g8 + 2 * c + kq) * cop + co0 + (lane & 31)];
        for (int tap = 0; tap < 27; ++tap) {
            s16x8 a1;
            if (tap + 1 < 27) a1 = wp[((size_t)(tap + 1) * g8 + 2 * c + kq) * cop + co0 + (lane & 31)];
            const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;  // offsets + 1
#pragma unroll
            for (int r = 0; r < RW; ++r)
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    const int hp = ((lz[r] + dz) * HY + (ly[r] + dy)) * kHX + 32 * s + (lane & 31) + dx;
                    const s16x8 b = sx[2 * hp + kq];
                    acc[r][s] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a0),
                                                                        __builtin_bit_cast(bf16x8, b), acc[r][s], 0, 0, 0);
                }
            a0 = a1;
        }
    }
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            if (!pok[r][s]) continue;
            const int p = ((z0 + lz[r]) * H + y0 + ly[r]) * W + x0 + 32 * s + (lane & 31);
            epilogue32(acc[r][s], p, P, co0, kq, cout, bias, skip, relu, Y, yb);
        }
}

// The same brick for layers of at most 16 output channels, on 16-row tiles
// (v_mfma_f32_16x16x32_bf16): lane l holds A[l % 16][k0 + 8 (l / 16) + j] and
// B[k0 + 8 (l / 16) + j][l % 16], and the accumulator element v of lane l is
// D[4 (l / 16) + v][l % 16].  A K step of 32 covers (tap, 8-channel half)
// pairs 4 t .. 4 t + 3 of the 16-channel block, i.e. two taps: 14 steps per
// block (the last half empty) instead of 27, and each weight load feeds the
// four 16-position tiles of the wave's row.
template <int BY, int BZ, int NW>
__global__ void __launch_bounds__(64 * NW)
    k_conv_bf16_lds16(const short* __restrict__ Xb, int cin, const uint32_t* __restrict__ packed,
                      const float* __restrict__ bias, const float* __restrict__ skip, float* __restrict__ Y,
                      short* __restrict__ yb, int cout, int D, int H, int W, int relu) {
    constexpr int HY = BY + 2, HALO = halo_positions<BY, BZ>();
    static_assert(BY * BZ == NW, "one row per wave");
    __shared__ __align__(16) s16x8 sx[HALO * 2];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int P = D * H * W;
    const int cip = cin_pad_of(cin, LBM_NN_BF16), cop = cout_pad_of(cout);
    const int nbx = (W + kBX - 1) / kBX, nby = (H + BY - 1) / BY;
    const int bx = blockIdx.x % nbx, by = (blockIdx.x / nbx) % nby, bz = blockIdx.x / (nbx * nby);
    const int x0 = bx * kBX, y0 = by * BY, z0 = bz * BZ;
    const int g = lane >> 4, col = lane & 15;
    const int ly = wave % BY, lz = wave / BY;
    const bool rok = y0 + ly < H && z0 + lz < D;
    f32x4 acc[4];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[s][v] = 0.0f;
    const s16x8* wp = reinterpret_cast<const s16x8*>(packed);
    const s16x8* xg = reinterpret_cast<const s16x8*>(Xb);
    const int g8 = cip / 8;
    const s16x8 zero = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int c = 0; c < cip / 16; ++c) {
        __syncthreads();
        for (int i = threadIdx.x; i < HALO * 2; i += 64 * NW) {
            const int hp = i >> 1, half = i & 1;
            const int hx = hp % kHX, hy = (hp / kHX) % HY, hz = hp / (kHX * HY);
            int gx = wrapc(x0 + hx - 1, W), gy = wrapc(y0 + hy - 1, H), gz = wrapc(z0 + hz - 1, D);
            gx = gx < W ? gx : gx % W;
            gy = gy < H ? gy : gy % H;
            gz = gz < D ? gz : gz % D;
            sx[i] = xg[((size_t)(gz * H + gy) * W + gx) * g8 + 2 * c + half];
        }
        __syncthreads();
        // this lane's (tap, half) of K step t is pair 4 t + g; pairs 54, 55 are empty
        auto wload = [&](int t) {
            const int pr = 4 * t + g;
            return pr < 54 ? wp[((size_t)(pr >> 1) * g8 + 2 * c + (pr & 1)) * cop + col] : zero;
        };
        s16x8 a0 = wload(0);
        for (int t = 0; t < 14; ++t) {
            s16x8 a1;
            if (t + 1 < 14) a1 = wload(t + 1);
            const int pr = 4 * t + g;
            const int tap = pr < 54 ? pr >> 1 : 26, half = pr & 1;
            const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;  // offsets + 1
            const int hrow = ((lz + dz) * HY + (ly + dy)) * kHX + dx + col;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const s16x8 b = sx[2 * (hrow + 16 * s) + half];
                acc[s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a0),
                                                                 __builtin_bit_cast(bf16x8, b), acc[s], 0, 0, 0);
            }
            a0 = a1;
        }
    }
    if (!rok) return;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int x = x0 + 16 * s + col;
        if (x >= W) continue;
        const int p = ((z0 + lz) * H + y0 + ly) * W + x;
        float r[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int co = 4 * g + v;
            r[v] = 0.0f;
            if (co < cout) {
                float t = acc[s][v] + (bias ? bias[co] : 0.0f);
                if (relu) t = t > 0.0f ? t : 0.0f;
                if (skip) t += skip[(size_t)co * P + p];
                r[v] = t;
                if (Y) Y[(size_t)co * P + p] = t;
            }
        }
        if (yb) store_yb4(yb, 16, p, 4 * g, cout, r);
    }
}

// Weight gradient partial tiles: one wave per (co block, n block, position chunk),
// n = ci * 27 + tap.
// FP32 -> BF16 (round to nearest even), elementwise.
__global__ void k_to_bf16(const float* __restrict__ x, short* __restrict__ y, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = f2bf(x[i]);
}

template <int PREC>
__global__ void __launch_bounds__(64)
    k_wgrad(const float* __restrict__ X, int cin, const float* __restrict__ dY, int cout, int D, int H, int W,
            int chunk, float* __restrict__ partial, const short* __restrict__ Xh, const short* __restrict__ dYh) {
    const int lane = threadIdx.x;
    const int P = D * H * W;
    const int co0 = blockIdx.x * 32, n0 = blockIdx.y * 32, ch = blockIdx.z;
    const int kq = lane >> 5;
    const int NN = cin * 27;
    const int m = co0 + (lane & 31);  // A row (co) of this lane
    const int n = n0 + (lane & 31);   // B column ((ci, tap)) of this lane
    const bool mok = m < cout, nok = n < NN;
    const int ci = nok ? n / 27 : 0, tap = nok ? n % 27 : 0;
    const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
    const int p0 = ch * chunk, p1 = (p0 + chunk < P) ? p0 + chunk : P;
    f32x16 acc;
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
    constexpr int KW = PREC == LBM_NN_BF16 ? 4 : 1;
    constexpr int KS = 2 * KW;
    for (int pk = p0; pk < p1; pk += KS) {
        float av[KW], bv[KW];
        [[maybe_unused]] bf16x4 ah, bh;
#pragma unroll
        for (int j = 0; j < KW; ++j) {
            const int p = pk + kq * KW + j;
            const bool ok = p < p1;
            const int pp = ok ? p : p0;
            const int x = pp % W, y = (pp / W) % H, z = pp / (W * H);
            const int q = (wrapc(z + dz, D) * H + wrapc(y + dy, H)) * W + wrapc(x + dx, W);
            if constexpr (PREC == LBM_NN_BF16) {
                // operands converted once by the launcher (same rounding)
                ah[j] = (ok && mok) ? dYh[(size_t)m * P + pp] : (short)0;
                bh[j] = (ok && nok) ? Xh[(size_t)ci * P + q] : (short)0;
            } else {
                av[j] = (ok && mok) ? dY[(size_t)m * P + pp] : 0.0f;
                bv[j] = (ok && nok) ? X[(size_t)ci * P + q] : 0.0f;
            }
        }
        if constexpr (PREC == LBM_NN_BF16) {
            acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(ah, bh, acc, 0, 0, 0);
        } else {
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[0], bv[0], acc, 0, 0, 0);
        }
    }
    // partial[ch][co][n] over the full (cout x NN) extent
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int co = co0 + 8 * (v / 4) + 4 * kq + (v % 4);
        const int nn = n0 + (lane & 31);
        if (co < cout && nn < NN) partial[((size_t)ch * cout + co) * NN + nn] = acc[v];
    }
}

// The same partial tiles from the BF16 copies with the gfx950 32x32x16 MFMA,
// for rows of a multiple of 8 positions: a lane half takes 8 consecutive
// positions of one row, so its dY operand is one aligned 16-byte load and
// its X operand, shifted by the tap's dx (periodic in x), is formed from two
// aligned 16-byte loads of the shifted row by a one-element funnel shift.
// The position coordinates are computed once per 8 positions.  chunk is a
// multiple of 16 and P of 8, so a half is wholly inside or outside [p0, p1).
__device__ __forceinline__ s16x8 load16(const short* p) { return *reinterpret_cast<const s16x8*>(p); }

__global__ void __launch_bounds__(64)
    k_wgrad_w8(const short* __restrict__ Xh, int cin, const short* __restrict__ dYh, int cout, int D, int H, int W,
               int chunk, float* __restrict__ partial) {
    const int lane = threadIdx.x;
    const int P = D * H * W;
    const int co0 = blockIdx.x * 32, n0 = blockIdx.y * 32, ch = blockIdx.z;
    const int kq = lane >> 5;
    const int NN = cin * 27;
    const int m = co0 + (lane & 31);
    const int n = n0 + (lane & 31);
    const bool mok = m < cout, nok = n < NN;
    const int ci = nok ? n / 27 : 0, tap = nok ? n % 27 : 0;
    const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
    const int p0 = ch * chunk, p1 = (p0 + chunk < P) ? p0 + chunk : P;
    const short* xrow = Xh + (size_t)ci * P;
    const short* yrow = dYh + (size_t)m * P;
    f32x16 acc;
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
    const s16x8 zero = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int pk = p0; pk < p1; pk += 16) {
        const int p = pk + 8 * kq;  // this half's 8 positions, one row
        s16x8 a = zero, b = zero;
        if (p < p1) {
            const int x0 = p % W, y = (p / W) % H, z = p / (W * H);
            if (mok) a = load16(yrow + p);
            if (nok) {
                const short* row = xrow + (size_t)(wrapc(z + dz, D) * H + wrapc(y + dy, H)) * W;
                const s16x8 cur = load16(row + x0);
                if (dx == 0) {
                    b = cur;
                } else {
                    // neighbouring run of the row (wrapping) and one-element shift
                    const int xo = dx > 0 ? (x0 + 8 == W ? 0 : x0 + 8) : (x0 == 0 ? W - 8 : x0 - 8);
                    const s16x8 nb = load16(row + xo);
                    if (dx > 0) {
                        b = __builtin_shufflevector(cur, nb, 1, 2, 3, 4, 5, 6, 7, 8);
                    } else {
                        b = __builtin_shufflevector(nb, cur, 7, 8, 9, 10, 11, 12, 13, 14);
                    }
                }
            }
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                       acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int co = co0 + 8 * (v / 4) + 4 * kq + (v % 4);
        const int nn = n0 + (lane & 31);
        if (co < cout && nn < NN) partial[((size_t)ch * cout + co) * NN + nn] = acc[v];
    }
}

__global__ void k_chunk_sum(const float* __restrict__ partial, int nchunk, int64_t n, float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.0f;
    for (int c = 0; c < nchunk; ++c) s += partial[(size_t)c * n + i];
    out[i] = s;
}

// Bias gradient in two fixed-order passes: block (j, c) sums chunk j of
// channel c in double, then one thread per channel adds the chunk sums.
constexpr int kBiasChunks = 64;
__global__ void __launch_bounds__(256) k_bias_partial(const float* __restrict__ dY, int64_t P,
                                                      double* __restrict__ part) {
    const int j = blockIdx.x, c = blockIdx.y;
    const int64_t per = (P + kBiasChunks - 1) / kBiasChunks;
    const int64_t p0 = j * per, p1 = p0 + per < P ? p0 + per : P;
    double s = 0.0;
    for (int64_t p = p0 + threadIdx.x; p < p1; p += 256) s += dY[(size_t)c * P + p];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    __shared__ double sh[4];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[(size_t)c * kBiasChunks + j] = sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ void k_bias_final(const double* __restrict__ part, int C, float* __restrict__ db) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < C; c += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int j = 0; j < kBiasChunks; ++j) s += part[(size_t)c * kBiasChunks + j];
        db[c] = (float)s;
    }
}

__global__ void k_relu_bwd(const float* __restrict__ Y, float* __restrict__ dY, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !(Y[i] > 0.0f)) dY[i] = 0.0f;
}

__global__ void k_add(float* __restrict__ y, const float* __restrict__ x, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] += x[i];
}

// coarse index (c, z, y, x) over [c][D/2][H/2][W/2]
__global__ void k_pool(const float* __restrict__ X, int c, int D, int H, int W, float* __restrict__ Y) {
    const int Dc = D / 2, Hc = H / 2, Wc = W / 2;
    const int64_t total = (int64_t)c * Dc * Hc * Wc;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int x = i % Wc, y = (i / Wc) % Hc, z = (i / ((int64_t)Wc * Hc)) % Dc;
    const int64_t ch = i / ((int64_t)Wc * Hc * Dc);
    const float* b = X + (size_t)ch * D * H * W;
    float s = 0.0f;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) s += b[((size_t)(2 * z + dz) * H + 2 * y + dy) * W + 2 * x + dx];
    Y[i] = 0.125f * s;
}

// fine index over [c][D][H][W]
__global__ void k_pool_bwd(const float* __restrict__ dY, int c, int D, int H, int W, float* __restrict__ dX,
                           int accumulate) {
    const int64_t total = (int64_t)c * D * H * W;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int x = i % W, y = (i / W) % H, z = (i / ((int64_t)W * H)) % D;
    const int64_t ch = i / ((int64_t)W * H * D);
    const float v = 0.125f * dY[(((size_t)ch * (D / 2) + z / 2) * (H / 2) + y / 2) * (W / 2) + x / 2];
    dX[i] = accumulate ? dX[i] + v : v;
}

// fine index over [c][2D][2H][2W], X coarse [c][D][H][W]
// One thread per coarse element: it writes its 2 x 2 x 2 fine copies as four
// 8-byte pairs (coalesced along x).
__global__ void k_up(const float* __restrict__ X, int c, int D, int H, int W, float* __restrict__ Y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)c * D * H * W) return;
    const int x = (int)(i % W), y = (int)((i / W) % H);
    const int64_t zc = i / ((int64_t)W * H);  // channel * D + z
    const float v = X[i];
    const float2 vv = make_float2(v, v);
    const int Wf = 2 * W, Hf = 2 * H;
#pragma unroll
    for (int dz = 0; dz < 2; ++dz)
#pragma unroll
        for (int dy = 0; dy < 2; ++dy) {
            const size_t row = ((size_t)(2 * zc + dz) * Hf + 2 * y + dy) * Wf;
            *reinterpret_cast<float2*>(Y + row + 2 * x) = vv;
        }
}

// Pooling and upsampling straight into the BF16 channels-innermost input of a
// convolution (the work layout: [P][c padded to 16], padding channels zero):
// the same values as k_pool / k_up followed by the conversion, without the
// FP32 tensor in between.  Like k_act_pack, a block transposes 64 output
// positions through LDS (coalesced reads of each channel, one contiguous run
// of 16-byte words written); MODE 0 pools 2x2x2 of the fine input X [c][D][H][W],
// MODE 1 copies the coarse parent of X [c][D][H][W] into the 2D x 2H x 2W grid.
template <int MODE>
__global__ void __launch_bounds__(256) k_resample_x(const float* __restrict__ X, int c, int D, int H, int W,
                                                    s16x8* __restrict__ xb) {
    __shared__ short sh[kPackMaxC][kPackPos + 2];
    const int Do = MODE == 0 ? D / 2 : 2 * D, Ho = MODE == 0 ? H / 2 : 2 * H, Wo = MODE == 0 ? W / 2 : 2 * W;
    const int64_t Po = (int64_t)Do * Ho * Wo;
    const int64_t p0 = (int64_t)blockIdx.x * kPackPos;
    const int t = threadIdx.x, lp = t % kPackPos;
    const int64_t po = p0 + lp;
    const bool ok = po < Po;
    const int64_t pp = ok ? po : 0;
    const int x = (int)(pp % Wo), y = (int)((pp / Wo) % Ho), z = (int)(pp / ((int64_t)Wo * Ho));
    const size_t P = (size_t)D * H * W;
    const int cip = cin_pad_of(c, LBM_NN_BF16), G = cip / 8;
    for (int cb = 0; cb < cip; cb += kPackMaxC) {
        const int nc = cip - cb < kPackMaxC ? cip - cb : kPackMaxC;
        if (cb > 0) __syncthreads();
        for (int cl = t / kPackPos; cl < nc; cl += 256 / kPackPos) {
            const int ch = cb + cl;
            short v = 0;
            if (ch < c && ok) {
                const float* b = X + (size_t)ch * P;
                if constexpr (MODE == 0) {
                    float sum = 0.0f;
                    for (int dz = 0; dz < 2; ++dz)
                        for (int dy = 0; dy < 2; ++dy)
                            for (int dx = 0; dx < 2; ++dx)
                                sum += b[((size_t)(2 * z + dz) * H + 2 * y + dy) * W + 2 * x + dx];
                    v = f2bf(0.125f * sum);
                } else {
                    v = f2bf(b[((size_t)(z / 2) * H + y / 2) * W + x / 2]);
                }
            }
            sh[cl][lp] = v;
        }
        __syncthreads();
        const int Gc = nc / 8;
        for (int w = t; w < kPackPos * Gc; w += 256) {
            const int pos = w / Gc, g = w % Gc;
            if (p0 + pos >= Po) continue;
            s16x8 v;
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = sh[8 * g + j][pos];
            xb[(size_t)(p0 + pos) * G + cb / 8 + g] = v;
        }
    }
}

// coarse index over [c][D][H][W], dY fine
__global__ void k_up_bwd(const float* __restrict__ dY, int c, int D, int H, int W, float* __restrict__ dX) {
    const int64_t total = (int64_t)c * D * H * W;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int x = i % W, y = (i / W) % H, z = (i / ((int64_t)W * H)) % D;
    const int64_t ch = i / ((int64_t)W * H * D);
    const int Wf = 2 * W, Hf = 2 * H, Df = 2 * D;
    const float* b = dY + (size_t)ch * Df * Hf * Wf;
    float s = 0.0f;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) s += b[((size_t)(2 * z + dz) * Hf + 2 * y + dy) * Wf + 2 * x + dx];
    dX[i] = s;
}

__global__ void __launch_bounds__(256)
    k_mse_partial(const float* __restrict__ Y, const float* __restrict__ T, const float* __restrict__ mask, int c,
                  int64_t P, double* __restrict__ part) {
    double s = 0.0, m = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < P; p += (int64_t)gridDim.x * 256) {
        const float mk = mask[p];
        m += mk;
        for (int ch = 0; ch < c; ++ch) {
            const double d = (double)Y[(size_t)ch * P + p] - (double)T[(size_t)ch * P + p];
            s += mk * d * d;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        s += __shfl_xor(s, o, 64);
        m += __shfl_xor(m, o, 64);
    }
    __shared__ double sh[2][4];
    if ((threadIdx.x & 63) == 0) {
        sh[0][threadIdx.x >> 6] = s;
        sh[1][threadIdx.x >> 6] = m;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3];
        part[2 * blockIdx.x + 1] = sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3];
    }
}

__global__ void k_mse_final(const double* __restrict__ part, int nblk, int c, double* __restrict__ loss,
                            double* __restrict__ msum) {
    if (threadIdx.x != 0) return;
    double s = 0.0, m = 0.0;
    for (int b = 0; b < nblk; ++b) {
        s += part[2 * b];
        m += part[2 * b + 1];
    }
    *msum = m;
    *loss = m > 0.0 ? s / (c * m) : 0.0;
}

__global__ void k_mse_grad(const float* __restrict__ Y, const float* __restrict__ T, const float* __restrict__ mask,
                           int c, int64_t P, const double* __restrict__ msum, float* __restrict__ dY) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)c * P) return;
    const int64_t p = i % P;
    const double m = *msum;
    dY[i] = m > 0.0 ? (float)(2.0 * mask[p] * ((double)Y[i] - (double)T[i]) / (c * m)) : 0.0f;
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       int64_t n, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Warm-start fields from a network output (lbm_nn_warm_fields): the pore
// mean of channel 3 by per-block partial sums in a fixed order, then one
// elementwise pass in double precision.
__global__ void k_pore_sum_partial(const float* __restrict__ X, const float* __restrict__ mask, int64_t P,
                                   double* __restrict__ part) {
    double s = 0.0, m = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < P; p += (int64_t)gridDim.x * 256) {
        const double mk = mask[p];
        m += mk;
        s += mk * (double)X[p];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        s += __shfl_xor(s, o, 64);
        m += __shfl_xor(m, o, 64);
    }
    __shared__ double sh[2][4];
    if ((threadIdx.x & 63) == 0) {
        sh[0][threadIdx.x >> 6] = s;
        sh[1][threadIdx.x >> 6] = m;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3];
        part[2 * blockIdx.x + 1] = sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3];
    }
}

__global__ void k_pore_sum_final(const double* __restrict__ part, int nblk, double* __restrict__ out) {
    if (threadIdx.x != 0) return;
    double s = 0.0, m = 0.0;
    for (int b = 0; b < nblk; ++b) {
        s += part[2 * b];
        m += part[2 * b + 1];
    }
    out[0] = s;
    out[1] = m;
}

struct WarmArgs {
    double c[4];
    double shift_x;
};

template <typename R>
__global__ void k_warm_fields(const float* __restrict__ Y, const float* __restrict__ mask, int64_t P, WarmArgs a,
                              const double* __restrict__ sums, R* __restrict__ rho0, R* __restrict__ u0) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const bool pore = mask[i] != 0.0f;
    const double mean_p = sums[1] > 0.0 ? sums[0] / sums[1] : 0.0;
    rho0[i] = pore ? (R)(1.0 + a.c[3] * ((double)Y[3 * P + i] - mean_p)) : (R)1;
    for (int d = 0; d < 3; ++d)
        u0[d * P + i] = pore ? (R)(a.c[d] * (double)Y[d * P + i] - (d == 0 ? a.shift_x : 0.0)) : (R)0;
}

inline int grid1(int64_t n, int b = 256) { return (int)((n + b - 1) / b); }
inline int ok(hipError_t e) { return e == hipSuccess ? LBM_OK : LBM_ERR_HIP; }

int wgrad_chunks(int64_t P) { return P >= 65536 ? 64 : (P >= 4096 ? 8 : 1); }

constexpr int kBiasNoallocMaxC = 1024;
constexpr int kMaxDevices = 64;

}  // namespace

// Library-owned scratch of lbm_nn_bias_grad_noalloc: the chunk partial sums
// of up to kBiasNoallocMaxC channels (512 KiB), one copy per device for the
// life of the process.  Host code never passes the symbol itself to a kernel
// (in host code it names a host-side stand-in); it uses the device address
// that hipGetSymbolAddress returns, looked up once per device.
static __device__ __align__(256) double scratch[kBiasChunks * kBiasNoallocMaxC];
static double* g_scratch_dev[kMaxDevices] = {};
static std::mutex g_scratch_mu;

static int bias_scratch_ptr(double** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return LBM_ERR_HIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return LBM_ERR_HIP;
        g_scratch_dev[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_dev[dev];
    return LBM_OK;
}


// Symmetry transform of a field X [C][D][H][W] (training-set augmentation):
// Y[c](r) = sign[c] * X[src[c]](g^-1 r) with g = periodic shift o axis flips o
// optional exchange of the D and H axes (needs D == H).
struct AugArgs {
    int src[8];
    float sign[8];
    int sz, sy, sx, fz, fy, fx, swap;
};
__global__ void k_augment(const float* __restrict__ X, float* __restrict__ Y, int C, int D, int H, int W,
                          AugArgs a) {
    const int64_t P = (int64_t)D * H * W;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)C * P) return;
    const int c = (int)(i / P);
    const int64_t p = i % P;
    const int x = (int)(p % W), y = (int)((p / W) % H), z = (int)(p / ((int64_t)W * H));
    // undo the shift, then the flips, then the exchange
    int zs = z - a.sz, ys = y - a.sy, xs = x - a.sx;
    zs = zs < 0 ? zs + D : zs;
    ys = ys < 0 ? ys + H : ys;
    xs = xs < 0 ? xs + W : xs;
    if (a.fz) zs = D - 1 - zs;
    if (a.fy) ys = H - 1 - ys;
    if (a.fx) xs = W - 1 - xs;
    if (a.swap) {
        const int t = zs;
        zs = ys;
        ys = t;
    }
    Y[i] = a.sign[c] * X[(int64_t)a.src[c] * P + ((int64_t)zs * H + ys) * W + xs];
}

extern "C" {

size_t lbm_nn_packed_words(int c_out, int c_in) {
    // enough for either precision and either orientation
    const int cmax = c_out > c_in ? c_out : c_in;
    const size_t a = (size_t)27 * cin_pad_of(cmax, LBM_NN_BF16) * cout_pad_of(cmax);
    return a;  // fp32: one word per entry; bf16: half a word per entry
}

int lbm_nn_pack(const float* W, int c_out, int c_in, int transpose, int prec, uint32_t* packed, void* stream) {
    if (!W || !packed || c_out < 1 || c_in < 1 || (prec != LBM_NN_BF16 && prec != LBM_NN_FP32)) return LBM_ERR_ARG;
    const int lo = transpose ? c_in : c_out, li = transpose ? c_out : c_in;
    const int total = 27 * cin_pad_of(li, prec) * cout_pad_of(lo);
    hipLaunchKernelGGL(k_pack, dim3(grid1(total)), dim3(256), 0, (hipStream_t)stream, W, c_out, c_in, transpose,
                       prec, packed);
    return ok(hipGetLastError());
}

size_t lbm_nn_conv_work_bytes(int c_in, int D, int H, int W, int prec) {
    if (prec != LBM_NN_BF16 || c_in < 1 || D < 1 || H < 1 || W < 1) return 0;
    return (size_t)D * H * W * cin_pad_of(c_in, prec) * 2;
}

}  // extern "C"

// BF16 convolution from the channels-innermost input Xb: the LDS-staged
// kernels for rows of 32 or more positions (16-row tiles up to 16 output
// channels), the global-operand kernel otherwise.
static hipError_t conv_bf16_launch(const short* Xb, int c_in, const uint32_t* packed, const float* bias,
                                   const float* skip, float* Y, short* yb, int c_out, int D, int H, int W, int relu,
                                   hipStream_t st) {
    const int64_t P = (int64_t)D * H * W;
#if LBM_NN_CONV_LDS
    if (W >= 32) {
        constexpr int BY = LBM_NN_BRICK_Y, BZ = LBM_NN_BRICK_Z, NW = LBM_NN_BRICK_WAVES;
        const unsigned nb = (unsigned)(((W + kBX - 1) / kBX) * ((H + BY - 1) / BY) * ((D + BZ - 1) / BZ));
#if LBM_NN_CONV_16ROW
        if constexpr (BY * BZ == NW) {
            if (c_out <= 16) {
                hipLaunchKernelGGL((k_conv_bf16_lds16<BY, BZ, NW>), dim3(nb), dim3(64 * NW), 0, st, Xb, c_in, packed,
                                   bias, skip, Y, yb, c_out, D, H, W, relu);
                return hipGetLastError();
            }
        }
#endif
        hipLaunchKernelGGL((k_conv_bf16_lds<BY, BZ, NW>), dim3(nb, (unsigned)((c_out + 31) / 32)), dim3(64 * NW), 0,
                           st, Xb, c_in, packed, bias, skip, Y, yb, c_out, D, H, W, relu);
        return hipGetLastError();
    }
#endif
    constexpr int NT = LBM_NN_CONV_NT;
    dim3 grid((unsigned)((P + 128 * NT - 1) / (128 * NT)), (unsigned)((c_out + 31) / 32));
    hipLaunchKernelGGL(k_conv_bf16<NT>, grid, dim3(256), 0, st, Xb, c_in, packed, bias, skip, Y, yb, c_out, D, H, W,
                       relu);
    return hipGetLastError();
}

static void act_pack_launch(const float* X, int c_in, int64_t P, void* work, hipStream_t st) {
    const int cip = cin_pad_of(c_in, LBM_NN_BF16);
    hipLaunchKernelGGL(k_act_pack, dim3((unsigned)((P + kPackPos - 1) / kPackPos)), dim3(256), 0, st, X, c_in, cip,
                       P, reinterpret_cast<s16x8*>(work));
}

extern "C" {

int lbm_nn_conv(const float* X, int c_in, const uint32_t* packed, const float* bias, const float* skip, float* Y,
                int c_out, int D, int H, int W, int relu, int prec, void* work, void* stream) {
    if (!X || !packed || !Y || c_in < 1 || c_out < 1 || D < 1 || H < 1 || W < 1) return LBM_ERR_ARG;
    const int64_t P = (int64_t)D * H * W;
    if (P * (c_in > c_out ? c_in : c_out) >= (1LL << 31)) return LBM_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    if (prec == LBM_NN_BF16) {
        if (!work) return LBM_ERR_ARG;
        act_pack_launch(X, c_in, P, work, st);
        return ok(conv_bf16_launch(reinterpret_cast<const short*>(work), c_in, packed, bias, skip, Y, nullptr, c_out,
                                   D, H, W, relu, st));
    } else if (prec == LBM_NN_FP32) {
        dim3 grid((unsigned)((P + 127) / 128), (unsigned)((c_out + 31) / 32));
        hipLaunchKernelGGL(k_conv_f32, grid, dim3(256), 0, st, X, c_in, packed, bias, skip, Y, c_out, D, H, W, relu);
    } else {
        return LBM_ERR_ARG;
    }
    return ok(hipGetLastError());
}

int lbm_nn_conv_x(const float* X, const void* xb, int c_in, const uint32_t* packed, const float* bias,
                  const float* skip, float* Y, void* yb_next, int c_out, int D, int H, int W, int relu, void* work,
                  void* stream) {
    if ((!X && !xb) || !packed || (!Y && !yb_next) || c_in < 1 || c_out < 1 || D < 1 || H < 1 || W < 1)
        return LBM_ERR_ARG;
    const int64_t P = (int64_t)D * H * W;
    if (P * (c_in > c_out ? c_in : c_out) >= (1LL << 31)) return LBM_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    if (!xb) {
        if (!work) return LBM_ERR_ARG;
        act_pack_launch(X, c_in, P, work, st);
        xb = work;
    }
    return ok(conv_bf16_launch(reinterpret_cast<const short*>(xb), c_in, packed, bias, skip, Y,
                               reinterpret_cast<short*>(yb_next), c_out, D, H, W, relu, st));
}

// partial buffer: FP32 tile partials, then (aligned) the BF16 copies of X and dY
static size_t wgrad_tiles_words(int c_out, int c_in, int64_t P) {
    return ((size_t)wgrad_chunks(P) * c_out * c_in * 27 + 63) / 64 * 64;
}

size_t lbm_nn_wgrad_partial_words(int c_out, int c_in, int D, int H, int W) {
    const int64_t P = (int64_t)D * H * W;
    return wgrad_tiles_words(c_out, c_in, P) + ((size_t)(c_in + c_out) * P + 1) / 2;
}

int lbm_nn_wgrad(const float* X, int c_in, const float* dY, int c_out, int D, int H, int W, float* dW,
                 float* partial, int prec, void* stream) {
    if (!X || !dY || !dW || !partial || c_in < 1 || c_out < 1) return LBM_ERR_ARG;
    const int64_t P = (int64_t)D * H * W;
    const int nch = wgrad_chunks(P);
    // rows of a multiple of 8 positions take the 16-position steps of k_wgrad_w8
    // (its 16-byte operand loads need the BF16 copies 16-byte aligned)
    const bool w8 = prec == LBM_NN_BF16 && W % 8 == 0 && (reinterpret_cast<uintptr_t>(partial) & 15u) == 0;
    const int KS = w8 ? 16 : (prec == LBM_NN_BF16 ? 8 : 2);
    int chunk = (int)((P + nch - 1) / nch);
    chunk = (chunk + KS - 1) / KS * KS;
    dim3 grid((unsigned)((c_out + 31) / 32), (unsigned)((c_in * 27 + 31) / 32), (unsigned)nch);
    hipStream_t st = (hipStream_t)stream;
    if (prec == LBM_NN_BF16) {
        short* Xh = reinterpret_cast<short*>(partial + wgrad_tiles_words(c_out, c_in, P));
        short* dYh = Xh + (size_t)c_in * P;
        hipLaunchKernelGGL(k_to_bf16, dim3(grid1((int64_t)c_in * P)), dim3(256), 0, st, X, Xh, (int64_t)c_in * P);
        hipLaunchKernelGGL(k_to_bf16, dim3(grid1((int64_t)c_out * P)), dim3(256), 0, st, dY, dYh,
                           (int64_t)c_out * P);
        if (w8)
            hipLaunchKernelGGL(k_wgrad_w8, grid, dim3(64), 0, st, (const short*)Xh, c_in, (const short*)dYh, c_out,
                               D, H, W, chunk, partial);
        else
            hipLaunchKernelGGL(k_wgrad<LBM_NN_BF16>, grid, dim3(64), 0, st, X, c_in, dY, c_out, D, H, W, chunk,
                               partial, (const short*)Xh, (const short*)dYh);
    } else if (prec == LBM_NN_FP32) {
        hipLaunchKernelGGL(k_wgrad<LBM_NN_FP32>, grid, dim3(64), 0, st, X, c_in, dY, c_out, D, H, W, chunk, partial,
                           (const short*)nullptr, (const short*)nullptr);
    } else {
        return LBM_ERR_ARG;
    }
    const int64_t n = (int64_t)c_out * c_in * 27;
    hipLaunchKernelGGL(k_chunk_sum, dim3(grid1(n)), dim3(256), 0, st, partial, nch, n, dW);
    return ok(hipGetLastError());
}

int lbm_nn_bias_grad(const float* dY, int c, int64_t P, float* db, double* scratch, void* stream) {
    if (!dY || !db || !scratch || c < 1 || c > 65535 || P < 1) return LBM_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_bias_partial, dim3(kBiasChunks, c), dim3(256), 0, st, dY, P, scratch);
    hipLaunchKernelGGL(k_bias_final, dim3((c + 127) / 128), dim3(128), 0, st, scratch, c, db);
    return ok(hipGetLastError());
}

int lbm_nn_bias_grad_noalloc(const float* dY, int c, int64_t P, float* db, void* stream) {
    if (!dY || !db || c < 1 || c > kBiasNoallocMaxC || P < 1) return LBM_ERR_ARG;
    double* scratch = nullptr;
    const int rc = bias_scratch_ptr(&scratch);
    if (rc != LBM_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_bias_partial, dim3(kBiasChunks, c), dim3(256), 0, st, dY, P, scratch);
    hipLaunchKernelGGL(k_bias_final, dim3((c + 127) / 128), dim3(128), 0, st, scratch, c, db);
    return ok(hipGetLastError());
}

int lbm_nn_relu_bwd(const float* Y, float* dY, int64_t n, void* stream) {
    hipLaunchKernelGGL(k_relu_bwd, dim3(grid1(n)), dim3(256), 0, (hipStream_t)stream, Y, dY, n);
    return ok(hipGetLastError());
}

int lbm_nn_add(float* y, const float* x, int64_t n, void* stream) {
    hipLaunchKernelGGL(k_add, dim3(grid1(n)), dim3(256), 0, (hipStream_t)stream, y, x, n);
    return ok(hipGetLastError());
}

int lbm_nn_pool_x(const float* X, int c, int D, int H, int W, void* xb, void* stream) {
    if (!X || !xb || c < 1 || D < 2 || H < 2 || W < 2 || ((D | H | W) & 1)) return LBM_ERR_ARG;
    const int64_t n = (int64_t)(D / 2) * (H / 2) * (W / 2);
    hipLaunchKernelGGL(k_resample_x<0>, dim3((unsigned)((n + kPackPos - 1) / kPackPos)), dim3(256), 0,
                       (hipStream_t)stream, X, c, D, H, W, reinterpret_cast<s16x8*>(xb));
    return ok(hipGetLastError());
}

int lbm_nn_up_x(const float* X, int c, int D, int H, int W, void* xb, void* stream) {
    if (!X || !xb || c < 1 || D < 1 || H < 1 || W < 1) return LBM_ERR_ARG;
    const int64_t n = (int64_t)8 * D * H * W;
    hipLaunchKernelGGL(k_resample_x<1>, dim3((unsigned)((n + kPackPos - 1) / kPackPos)), dim3(256), 0,
                       (hipStream_t)stream, X, c, D, H, W, reinterpret_cast<s16x8*>(xb));
    return ok(hipGetLastError());
}

int lbm_nn_pool(const float* X, int c, int D, int H, int W, float* Y, void* stream) {
    if ((D | H | W) & 1) return LBM_ERR_ARG;
    const int64_t n = (int64_t)c * (D / 2) * (H / 2) * (W / 2);
    hipLaunchKernelGGL(k_pool, dim3(grid1(n)), dim3(256), 0, (hipStream_t)stream, X, c, D, H, W, Y);
    return ok(hipGetLastError());
}

int lbm_nn_pool_bwd(const float* dY, int c, int D, int H, int W, float* dX, int accumulate, void* stream) {
    if ((D | H | W) & 1) return LBM_ERR_ARG;
    const int64_t n = (int64_t)c * D * H * W;
    hipLaunchKernelGGL(k_pool_bwd, dim3(grid1(n)), dim3(256), 0, (hipStream_t)stream, dY, c, D, H, W, dX, accumulate);
    return ok(hipGetLastError());
}

int lbm_nn_up(const float* X, int c, int D, int H, int W, float* Y, void* stream) {
    const int64_t n = (int64_t)c * D * H * W;
    hipLaunchKernelGGL(k_up, dim3(grid1(n)), dim3(256), 0, (hipStream_t)stream, X, c, D, H, W, Y);
    return ok(hipGetLastError());
}

int lbm_nn_up_bwd(const float* dY, int c, int D, int H, int W, float* dX, void* stream) {
    const int64_t n = (int64_t)c * D * H * W;
    hipLaunchKernelGGL(k_up_bwd, dim3(grid1(n)), dim3(256), 0, (hipStream_t)stream, dY, c, D, H, W, dX);
    return ok(hipGetLastError());
}

int lbm_nn_mse(const float* Y, const float* T, const float* mask, int c, int64_t P, double* loss, float* dY,
               void* stream) {
    if (!Y || !T || !mask || !loss || c < 1 || P < 1) return LBM_ERR_ARG;
    // loss[0] = L, loss[1..] scratch: caller provides 2 + 2*256 doubles
    hipStream_t st = (hipStream_t)stream;
    const int nblk = 256;
    hipLaunchKernelGGL(k_mse_partial, dim3(nblk), dim3(256), 0, st, Y, T, mask, c, P, loss + 2);
    hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(64), 0, st, loss + 2, nblk, c, loss, loss + 1);
    if (dY)
        hipLaunchKernelGGL(k_mse_grad, dim3(grid1((int64_t)c * P)), dim3(256), 0, st, Y, T, mask, c, P, loss + 1, dY);
    return ok(hipGetLastError());
}

int lbm_nn_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float beta1, float beta2,
                float eps, int t, void* stream) {
    if (!p || !g || !m || !v || t < 1) return LBM_ERR_ARG;
    const float c1 = 1.0f - powf(beta1, (float)t), c2 = 1.0f - powf(beta2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3(grid1(n)), dim3(256), 0, (hipStream_t)stream, p, g, m, v, n, lr, beta1, beta2,
                       eps, c1, c2);
    return ok(hipGetLastError());
}

int lbm_nn_warm_fields(const float* Y, const float* mask, int64_t P, const double* c, double shift_x,
                       int real_bytes, void* rho0, void* u0, double* scratch, void* stream) {
    if (!Y || !mask || !c || !rho0 || !u0 || !scratch || P < 1 || (real_bytes != 4 && real_bytes != 8))
        return LBM_ERR_ARG;
    hipStream_t st = (hipStream_t)stream;
    const int nblk = 256;
    hipLaunchKernelGGL(k_pore_sum_partial, dim3(nblk), dim3(256), 0, st, Y + 3 * P, mask, P, scratch + 2);
    hipLaunchKernelGGL(k_pore_sum_final, dim3(1), dim3(64), 0, st, scratch + 2, nblk, scratch);
    WarmArgs a{};
    for (int k = 0; k < 4; ++k) a.c[k] = c[k];
    a.shift_x = shift_x;
    if (real_bytes == 8)
        hipLaunchKernelGGL(k_warm_fields<double>, dim3(grid1(P)), dim3(256), 0, st, Y, mask, P, a, scratch,
                           (double*)rho0, (double*)u0);
    else
        hipLaunchKernelGGL(k_warm_fields<float>, dim3(grid1(P)), dim3(256), 0, st, Y, mask, P, a, scratch,
                           (float*)rho0, (float*)u0);
    return ok(hipGetLastError());
}

int lbm_nn_augment(const float* X, float* Y, int c, int D, int H, int W, const int* shift, const int* flip,
                   int swap, const int* src, const float* sign, void* stream) {
    if (!X || !Y || !shift || !flip || !src || !sign || c < 1 || c > 8 || D < 1 || H < 1 || W < 1)
        return LBM_ERR_ARG;
    if (swap && D != H) return LBM_ERR_ARG;
    AugArgs a{};
    for (int k = 0; k < c; ++k) {
        if (src[k] < 0 || src[k] >= c) return LBM_ERR_ARG;
        a.src[k] = src[k];
        a.sign[k] = sign[k];
    }
    const int dims[3] = {D, H, W};
    int sh[3];
    for (int d = 0; d < 3; ++d) {
        sh[d] = shift[d] % dims[d];
        if (sh[d] < 0) sh[d] += dims[d];
    }
    a.sz = sh[0];
    a.sy = sh[1];
    a.sx = sh[2];
    a.fz = flip[0] != 0;
    a.fy = flip[1] != 0;
    a.fx = flip[2] != 0;
    a.swap = swap != 0;
    const int64_t n = (int64_t)c * D * H * W;
    hipLaunchKernelGGL(k_augment, dim3(grid1(n)), dim3(256), 0, (hipStream_t)stream, X, Y, c, D, H, W, a);
    return ok(hipGetLastError());
}

}  // extern "C"
