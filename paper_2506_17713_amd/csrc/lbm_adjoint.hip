// Hand-written reverse-mode adjoint of the fused step (one fluid component,
// FP32 or FP64 populations, D2Q9 or D3Q19, BGK or MRT).
//
// Forward map of one step, state s_t = post-collision populations f*(t-1):
//   f(x)    = s_i(x - e_i), or s_opp(i)(x) when x - e_i is solid      (pull)
//   rho, j  = sum_i f_i, sum_i f_i e_i                                 (Eq. 4)
//   rho_s   = clamp(phi rho_ave) or clamp(rho_ave - drho) at solids    (Eq. 17)
//   psi, U  = EOS pseudopotential of rho (fluid) or rho_s (solid)      (Eq. 12)
//   F(x)    = -A sum_i G_i U(x+e_i) e_i - (1-A) g psi(x) sum_i G_i psi(x+e_i) e_i + rho a   (Eq. 13)
//   f*(x)   = f - K (f - feq(rho, u)) + feq(rho, u + F/rho) - feq(rho, u),  u = j/rho      (Eq. 3, 5)
// with K = omega I (BGK) or M^T D^-1 S M (MRT; symmetric).  The adjoint runs
// these in reverse for every step, recomputing the forward fields from the
// state, which is rebuilt segment by segment from checkpoints.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "lbm_internal.hpp"

using namespace lbm;
using namespace lbmi;

namespace {

template <class R>
struct AdjArgs {
    const void* s;        // forward state s_t [Q][N]
    const uint32_t* nbr;  // neighbour words [N]
    const R* wet;         // wetting parameter [N]
    R* rho;               // fluid density, -1 at solids [N]
    R* rhoe;              // density fed to the EOS (rho or rho_s) [N]
    R* psi;               // [N]
    R* U;                 // [N]
    R* rave;              // rho_ave at active solids [N]
    R* wsum;              // sum of fluid-neighbour weights at active solids [N]
    uint8_t* flag;        // 0 inactive solid, 1 fluid, 2 active solid, 3 active solid at a limit
    const R* lam_in;      // adjoint of s_{t+1} [Q][N]
    R* lam_out;           // adjoint of s_t [Q][N]
    R* fbar;              // adjoint of the pulled populations (local part) [Q][N]
    R* Fbar;              // adjoint of the force [3][N]
    R* pbar_own;          // adjoint of psi(x) through its own force term [N]
    R* rbar_e;            // adjoint of rho at fluid nodes through psi/U [N]
    R* rbar_ave;          // adjoint of rho_ave at active solids [N]
    double* dwet;         // accumulated dL/d(wetting parameter) [N]
    double* tacc;         // accumulated dL/dT contributions [N]
    double* lpart;        // observable partial sums [blocks]
    const R* dLdrho;      // custom observable gradient [N]
    int NA, NB, NCc, N;
    R omega;
    R srate[19];
    R eos_a, eos_b, eos_R, eos_T, alpha, ginv, A, g;
    R body[3];
    R rho_min, rho_max;
    int psi_cs, wet_drho, obs;
    R rho_mid, inv_delta, inv_npore;
};

__device__ __forceinline__ int wrap1(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

template <int LAT>
__device__ __forceinline__ void decode(int n, int NA, int NB, int& a, int& b, int& c) {
    a = n % NA;
    const int t = n / NA;
    b = t % NB;
    c = t / NB;
}

template <int LAT>
__device__ __forceinline__ int shift(int a, int b, int c, int da, int db, int dc, int NA, int NB, int NCc) {
    return (wrap1(c + dc, NCc) * NB + wrap1(b + db, NB)) * NA + wrap1(a + da, NA);
}

// f(x) of the forward pull from state s (layout [Q][N]).
template <int LAT, class R>
__device__ __forceinline__ void pull_plain(const R* s, int n, int a, int b, int c, uint32_t word, int NA,
                                           int NB, int NCc, int N, R (&f)[Lat<LAT>::Q]) {
    using L = Lat<LAT>;
    sfor<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int o = opp(i);
        if (i != 0 && ((word >> i) & 1u)) {
            f[i] = s[(size_t)o * N + n];
        } else {
            const int m = shift<LAT>(a, b, c, -L::ea(i), -L::eb(i), -L::ec(i), NA, NB, NCc);
            f[i] = s[(size_t)i * N + m];
        }
    });
}

template <class R>
__device__ __forceinline__ void eos(const AdjArgs<R>& P, R rho, R& psi, R& U, R& dpsi, R& dU, R& psiT, R& UT) {
    if (P.psi_cs) {
        const R eta = P.eos_b * rho * (R)0.25;
        const R om = (R)1 - eta;
        const R om3 = om * om * om;
        const R Z = ((R)1 + eta + eta * eta - eta * eta * eta) / om3;
        // dZ/deta = [(1 + 2eta - 3eta^2)(1 - eta) + 3(1 + eta + eta^2 - eta^3)] / (1 - eta)^4
        const R dZ = (((R)1 + (R)2 * eta - (R)3 * eta * eta) * om +
                      (R)3 * ((R)1 + eta + eta * eta - eta * eta * eta)) / (om3 * om);
        const R RT = P.eos_R * P.eos_T;
        const R p = rho * RT * Z - P.eos_a * rho * rho;
        const R dp = RT * Z + rho * RT * dZ * P.eos_b * (R)0.25 - (R)2 * P.eos_a * rho;
        U = P.alpha * p - rho * (R)(1.0 / 3.0);
        dU = P.alpha * dp - (R)(1.0 / 3.0);
        UT = P.alpha * rho * P.eos_R * Z;
        R arg = (R)2 * U * P.ginv;
        if (arg > (R)0) {
            psi = sqrt(arg);
            dpsi = dU * P.ginv / psi;
            psiT = UT * P.ginv / psi;
        } else {
            psi = 0;
            dpsi = 0;
            psiT = 0;
        }
    } else {
        psi = rho;
        U = 0;
        dpsi = 1;
        dU = 0;
        psiT = 0;
        UT = 0;
    }
}

// --- forward fields -------------------------------------------------------
template <int LAT, class R>
__global__ void k_adj_rho(AdjArgs<R> P) {
    using L = Lat<LAT>;
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= P.N) return;
    const uint32_t w = P.nbr[n];
    if (w & 1u) {
        P.rho[n] = (R)-1;
        return;
    }
    int a, b, c;
    decode<LAT>(n, P.NA, P.NB, a, b, c);
    R f[L::Q];
    pull_plain<LAT>(reinterpret_cast<const R*>(P.s), n, a, b, c, w, P.NA, P.NB, P.NCc, P.N, f);
    R r = 0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) r += f[i];
    P.rho[n] = r;
}

template <int LAT, class R>
__global__ void k_adj_psi(AdjArgs<R> P) {
    using L = Lat<LAT>;
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= P.N) return;
    const uint32_t w = P.nbr[n];
    R re;
    uint8_t fl;
    if (!(w & 1u)) {
        re = P.rho[n];
        fl = 1;
    } else {
        int a, b, c;
        decode<LAT>(n, P.NA, P.NB, a, b, c);
        R num = 0, den = 0;
        sfor<L::Q - 1>([&](auto I) {
            constexpr int i = decltype(I)::value + 1;
            const int m = shift<LAT>(a, b, c, L::ea(i), L::eb(i), L::ec(i), P.NA, P.NB, P.NCc);
            const R r = P.rho[m];
            if (r >= (R)0) {
                den += (R)L::w(i);
                num += (R)L::w(i) * r;
            }
        });
        if (den == (R)0) {
            P.flag[n] = 0;
            P.rhoe[n] = 0;
            P.psi[n] = 0;
            P.U[n] = 0;
            return;
        }
        const R ra = num / den;
        const R prm = P.wet[n];
        R rs = P.wet_drho ? ra - prm : prm * ra;
        fl = 2;
        if (rs < P.rho_min) {
            rs = P.rho_min;
            fl = 3;
        }
        if (rs > P.rho_max) {
            rs = P.rho_max;
            fl = 3;
        }
        re = rs;
        P.rave[n] = ra;
        P.wsum[n] = den;
    }
    R ps, u, d1, d2, d3, d4;
    eos(P, re, ps, u, d1, d2, d3, d4);
    P.flag[n] = fl;
    P.rhoe[n] = re;
    P.psi[n] = ps;
    P.U[n] = u;
}

// --- collision + forcing adjoint (pointwise) --------------------------------
// G(c, v) = sum_i c_i d feq_i / dv = sum_i c_i w_i rho (3 e_i + 9 (e_i.v) e_i - 3 v)
template <int LAT, class R>
__device__ __forceinline__ void feq_grad(const R (&cf)[Lat<LAT>::Q], R rho, R vx, R vy, R vz, R& gx, R& gy,
                                         R& gz, R& grho) {
    using L = Lat<LAT>;
    R sx = 0, sy = 0, sz = 0, s0 = 0, sr = 0;
    const R vsq = (R)1.5 * (vx * vx + vy * vy + vz * vz);
    sfor<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr R ex = L::ex[i], ey = L::ey[i], ez = L::ez[i];
        const R cw = cf[i] * (R)L::w(i);
        const R ev = ex * vx + ey * vy + ez * vz;
        const R t = cw * ((R)3 + (R)9 * ev);
        sx += t * ex;
        sy += t * ey;
        sz += t * ez;
        s0 += cw;
        sr += cw * ((R)1 + (R)3 * ev + (R)4.5 * ev * ev - vsq);  // feq_i / (w_i rho)
    });
    gx = rho * (sx - (R)3 * s0 * vx);
    gy = rho * (sy - (R)3 * s0 * vy);
    gz = rho * (sz - (R)3 * s0 * vz);
    grho = sr;  // d/drho of sum_i c_i feq_i
}

template <int LAT, class R, int COLL>
__global__ void k_adj_collide(AdjArgs<R> P) {
    using L = Lat<LAT>;
    constexpr int Q = L::Q;
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= P.N) return;
    const uint32_t w = P.nbr[n];
    if (w & 1u) return;
    int a, b, c;
    decode<LAT>(n, P.NA, P.NB, a, b, c);
    const size_t N = (size_t)P.N;
    R f[Q];
    pull_plain<LAT>(reinterpret_cast<const R*>(P.s), n, a, b, c, w, P.NA, P.NB, P.NCc, P.N, f);
    R rho = 0, jx = 0, jy = 0, jz = 0;
    sfor<Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        rho += f[i];
        jx += (R)L::ex[i] * f[i];
        jy += (R)L::ey[i] * f[i];
        jz += (R)L::ez[i] * f[i];
    });
    // force at x from the recomputed psi / U fields
    R Sx = 0, Sy = 0, Sz = 0, Zx = 0, Zy = 0, Zz = 0;
    sfor<Q - 1>([&](auto I) {
        constexpr int i = decltype(I)::value + 1;
        constexpr R G = (R)(3.0 * L::w(i));
        const int m = shift<LAT>(a, b, c, L::ea(i), L::eb(i), L::ec(i), P.NA, P.NB, P.NCc);
        const R ps = G * P.psi[m], uu = G * P.U[m];
        Sx += ps * (R)L::ex[i];
        Sy += ps * (R)L::ey[i];
        Sz += ps * (R)L::ez[i];
        Zx += uu * (R)L::ex[i];
        Zy += uu * (R)L::ey[i];
        Zz += uu * (R)L::ez[i];
    });
    const R psx = P.psi[n];
    const R Bk = (R)1 - P.A;
    const R Fx = -P.A * Zx - Bk * P.g * psx * Sx + rho * P.body[0];
    const R Fy = -P.A * Zy - Bk * P.g * psx * Sy + rho * P.body[1];
    const R Fz = -P.A * Zz - Bk * P.g * psx * Sz + rho * P.body[2];
    const R ir = (R)1 / rho;
    const R ux = jx * ir, uy = jy * ir, uz = jz * ir;
    const R vx = ux + Fx * ir, vy = uy + Fy * ir, vz = uz + Fz * ir;

    R lam[Q], Kl[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) lam[i] = P.lam_in[(size_t)i * N + n];
    if constexpr (COLL == COLL_BGK) {
#pragma unroll
        for (int i = 0; i < Q; ++i) Kl[i] = P.omega * lam[i];
    } else {
        R m[Q];
        sfor<Q>([&](auto M) {
            constexpr int mm = decltype(M)::value;
            R s = 0;
            sfor<Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                constexpr double cf = mrt_coef<LAT>(mm, i);
                if constexpr (cf != 0.0) s += (R)cf * lam[i];
            });
            m[mm] = s * P.srate[mm];
        });
        sfor<Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            R s = 0;
            sfor<Q>([&](auto M) {
                constexpr int mm = decltype(M)::value;
                constexpr double cf = mrt_coef<LAT>(mm, i);
                if constexpr (cf != 0.0) s += (R)cf * m[mm];
            });
            Kl[i] = s;
        });
    }
    // f* = (I - K) f + (K - I) feq(u) + feq(v):  c1 = K lam - lam on feq(u), c2 = lam on feq(v)
    R c1[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) c1[i] = Kl[i] - lam[i];
    R g1x, g1y, g1z, g1r, g2x, g2y, g2z, g2r;
    feq_grad<LAT>(c1, rho, ux, uy, uz, g1x, g1y, g1z, g1r);
    feq_grad<LAT>(lam, rho, vx, vy, vz, g2x, g2y, g2z, g2r);
    // v = u + F / rho
    const R Fbx = g2x * ir, Fby = g2y * ir, Fbz = g2z * ir;
    R rbar = g1r + g2r - (g2x * Fx + g2y * Fy + g2z * Fz) * ir * ir;
    const R ubx = g1x + g2x, uby = g1y + g2y, ubz = g1z + g2z;
    // u = j / rho
    const R jbx = ubx * ir, jby = uby * ir, jbz = ubz * ir;
    rbar -= (ubx * ux + uby * uy + ubz * uz) * ir;
    // body force rho a
    rbar += Fbx * P.body[0] + Fby * P.body[1] + Fbz * P.body[2];
    sfor<Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        P.fbar[(size_t)i * N + n] = lam[i] - Kl[i] + rbar + jbx * (R)L::ex[i] + jby * (R)L::ey[i] + jbz * (R)L::ez[i];
    });
    P.Fbar[n] = Fbx;
    P.Fbar[N + n] = Fby;
    P.Fbar[2 * N + n] = Fbz;
    P.pbar_own[n] = -Bk * P.g * (Fbx * Sx + Fby * Sy + Fbz * Sz);
}

// --- pseudopotential / virtual-density adjoint -------------------------------
template <int LAT, class R>
__global__ void k_adj_psi_bar(AdjArgs<R> P) {
    using L = Lat<LAT>;
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= P.N) return;
    const uint8_t fl = P.flag[n];
    const size_t N = (size_t)P.N;
    if (fl == 0) {
        P.rbar_e[n] = 0;
        P.rbar_ave[n] = 0;
        return;
    }
    int a, b, c;
    decode<LAT>(n, P.NA, P.NB, a, b, c);
    R pb = fl == 1 ? P.pbar_own[n] : (R)0, ub = 0;
    const R Bk = (R)1 - P.A;
    sfor<L::Q - 1>([&](auto I) {
        constexpr int i = decltype(I)::value + 1;
        constexpr R G = (R)(3.0 * L::w(i));
        // x = n - e_i sees n as its neighbour in direction i
        const int m = shift<LAT>(a, b, c, -L::ea(i), -L::eb(i), -L::ec(i), P.NA, P.NB, P.NCc);
        if (P.flag[m] == 1) {
            const R Fd = (R)L::ex[i] * P.Fbar[m] + (R)L::ey[i] * P.Fbar[N + m] + (R)L::ez[i] * P.Fbar[2 * N + m];
            pb += -Bk * P.g * P.psi[m] * G * Fd;
            ub += -P.A * G * Fd;
        }
    });
    R ps, u, dps, du, psT, uT;
    eos(P, P.rhoe[n], ps, u, dps, du, psT, uT);
    const R rb = pb * dps + ub * du;
    P.tacc[n] += (double)(pb * psT + ub * uT);
    if (fl == 1) {
        P.rbar_e[n] = rb;
        P.rbar_ave[n] = 0;
    } else if (fl == 2) {
        P.rbar_e[n] = 0;
        P.dwet[n] += (double)(rb * (P.wet_drho ? (R)-1 : P.rave[n]));
        P.rbar_ave[n] = rb * (P.wet_drho ? (R)1 : P.wet[n]);
    } else {
        P.rbar_e[n] = 0;
        P.rbar_ave[n] = 0;
    }
}

// --- density adjoint and reverse streaming -----------------------------------
template <int LAT, class R>
__global__ void k_adj_stream(AdjArgs<R> P) {
    using L = Lat<LAT>;
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= P.N) return;
    const uint32_t w = P.nbr[n];
    if (w & 1u) return;
    int a, b, c;
    decode<LAT>(n, P.NA, P.NB, a, b, c);
    const size_t N = (size_t)P.N;
    R rb = P.rbar_e[n];
    // only a solid neighbour x + e_i (bit opp(i) of the word) can be an active
    // solid, so fluid neighbours are not looked up
    sfor<L::Q - 1>([&](auto I) {
        constexpr int i = decltype(I)::value + 1;
        if ((w >> opp(i)) & 1u) {
            const int m = shift<LAT>(a, b, c, L::ea(i), L::eb(i), L::ec(i), P.NA, P.NB, P.NCc);
            if (P.flag[m] == 2) rb += P.rbar_ave[m] * (R)L::w(i) / P.wsum[m];
        }
    });
    sfor<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int o = opp(i);
        const R v = P.fbar[(size_t)i * N + n] + rb;
        if (i != 0 && ((w >> i) & 1u)) {
            P.lam_out[(size_t)o * N + n] = v;
        } else {
            const int m = shift<LAT>(a, b, c, -L::ea(i), -L::eb(i), -L::ec(i), P.NA, P.NB, P.NCc);
            P.lam_out[(size_t)i * N + m] = v;
        }
    });
}

// --- observable: value and seed of the adjoint at the final state -----------
template <int LAT, class R>
__global__ void __launch_bounds__(256) k_adj_seed(AdjArgs<R> P) {
    using L = Lat<LAT>;
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    double lv = 0.0;
    if (n < P.N) {
        const uint32_t w = P.nbr[n];
        if (!(w & 1u)) {
            int a, b, c;
            decode<LAT>(n, P.NA, P.NB, a, b, c);
            R f[L::Q];
            pull_plain<LAT>(reinterpret_cast<const R*>(P.s), n, a, b, c, w, P.NA, P.NB, P.NCc, P.N, f);
            R rho = 0;
#pragma unroll
            for (int i = 0; i < L::Q; ++i) rho += f[i];
            R d;
            if (P.obs == 0) {
                // smooth non-wetting (vapour) saturation: sigma((rho_mid - rho) / delta)
                const R z = (P.rho_mid - rho) * P.inv_delta;
                const R sg = (R)1 / ((R)1 + exp(-z));
                lv = (double)(sg * P.inv_npore);
                d = -sg * ((R)1 - sg) * P.inv_delta * P.inv_npore;
            } else {
                d = P.dLdrho[n];
                lv = (double)(d * rho);
            }
            const size_t N = (size_t)P.N;
            sfor<L::Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                constexpr int o = opp(i);
                if (i != 0 && ((w >> i) & 1u)) {
                    P.lam_out[(size_t)o * N + n] = d;
                } else {
                    const int m = shift<LAT>(a, b, c, -L::ea(i), -L::eb(i), -L::ec(i), P.NA, P.NB, P.NCc);
                    P.lam_out[(size_t)i * N + m] = d;
                }
            });
        }
    }
    // block sum of the observable (fixed order)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) lv += __shfl_xor(lv, o, 64);
    __shared__ double sh[4];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = lv;
    __syncthreads();
    if (threadIdx.x == 0) P.lpart[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ void k_sum_fixed(const double* __restrict__ x, int n, double* __restrict__ out) {
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += 64) v += x[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (threadIdx.x == 0) *out = v;
}

// First pass of a fixed-order sum of n values: block b adds the values
// [b * per, (b + 1) * per) (lane-strided, then a fixed shuffle tree and the
// waves in order) into part[b].  k_sum_fixed over part completes the sum; the
// result does not depend on scheduling.
constexpr int kSumBlocks = 512;
__global__ void __launch_bounds__(256) k_sum_partial(const double* __restrict__ x, int n, int per,
                                                     double* __restrict__ part) {
    __shared__ double s_w[4];
    const int lo = blockIdx.x * per;
    const int hi = lo + per < n ? lo + per : n;
    double v = 0.0;
    for (int i = lo + (int)threadIdx.x; i < hi; i += 256) v += x[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = ((s_w[0] + s_w[1]) + s_w[2]) + s_w[3];
}

// ---------------------------------------------------------------------------
// Workspace of lbm_grad (caller-owned).
// ---------------------------------------------------------------------------
struct GradLayout {
    size_t ckpt, seg, lamA, lamB, fbar, Fbar, rho, rhoe, psi, U, rave, wsum, pbar, rbe, rba, flag, tacc, lpart,
        tpart, sums, total;
    size_t state;
    int nseg, K;
};

GradLayout grad_layout(const lbm_handle* h, const lbm_grad_req* r) {
    GradLayout g{};
    const size_t N = h->N, q = q_of(h->p.lattice), rb = real_bytes(h->p.storage);
    g.state = q * N * rb;
    g.K = r->ckpt_every;
    g.nseg = (r->nsteps + g.K - 1) / g.K;
    size_t off = 0;
    auto take = [&](size_t b) {
        size_t o = off;
        off += align256(b);
        return o;
    };
    g.ckpt = take(g.state * (size_t)g.nseg);
    g.seg = take(g.state * (size_t)g.K);
    g.lamA = take(q * N * rb);
    g.lamB = take(q * N * rb);
    g.fbar = take(q * N * rb);
    g.Fbar = take(3 * N * rb);
    g.rho = take(N * rb);
    g.rhoe = take(N * rb);
    g.psi = take(N * rb);
    g.U = take(N * rb);
    g.rave = take(N * rb);
    g.wsum = take(N * rb);
    g.pbar = take(N * rb);
    g.rbe = take(N * rb);
    g.rba = take(N * rb);
    g.flag = take(N);
    g.tacc = take(N * 8);
    g.lpart = take(((N + 255) / 256) * 8);
    g.tpart = take(kSumBlocks * 8);
    g.sums = take(64);
    g.total = off;
    return g;
}

int check_req(const lbm_handle* h, const lbm_grad_req* r) {
    if (!h || !r) return LBM_ERR_ARG;
    if (r->nsteps < 1 || r->ckpt_every < 1 || r->reserved != 0) return LBM_ERR_ARG;
    if (r->observable != LBM_OBS_SATURATION && r->observable != LBM_OBS_DRHO) return LBM_ERR_ARG;
    if (r->observable == LBM_OBS_SATURATION && !(r->delta > 0.0)) return LBM_ERR_ARG;
    if (r->observable == LBM_OBS_DRHO && !r->dL_drho) return LBM_ERR_ARG;
    if (h->p.n_comp != 1) return LBM_ERR_UNSUPPORTED;
    if (h->p.storage != LBM_STORE_F32 && h->p.storage != LBM_STORE_F64) return LBM_ERR_UNSUPPORTED;
    if (h->p.kappa[0] != 0.0 || h->p.collision == LBM_CLBM || h->has_res || h->p.layout == LBM_LAYOUT_FLUID)
        return LBM_ERR_UNSUPPORTED;
    return LBM_OK;
}

template <int LAT, class R, int COLL>
int grad_impl(lbm_handle* h, const lbm_grad_req* r, double* L_out, double* dwet, double* dT_out) {
    const GradLayout G = grad_layout(h, r);
    char* gw = (char*)r->ws;
    const lbm_params& p = h->p;
    const int N = h->N;
    const int blk = 256, grid = (N + blk - 1) / blk;
    hipStream_t st = h->stream;
    hipError_t e = hipSuccess;

    AdjArgs<R> A;
    std::memset(&A, 0, sizeof(A));
    A.nbr = reinterpret_cast<const uint32_t*>(h->ws + h->lay.nbr);
    A.wet = reinterpret_cast<const R*>(h->ws + h->lay.wet);
    A.rho = (R*)(gw + G.rho);
    A.rhoe = (R*)(gw + G.rhoe);
    A.psi = (R*)(gw + G.psi);
    A.U = (R*)(gw + G.U);
    A.rave = (R*)(gw + G.rave);
    A.wsum = (R*)(gw + G.wsum);
    A.flag = (uint8_t*)(gw + G.flag);
    A.fbar = (R*)(gw + G.fbar);
    A.Fbar = (R*)(gw + G.Fbar);
    A.pbar_own = (R*)(gw + G.pbar);
    A.rbar_e = (R*)(gw + G.rbe);
    A.rbar_ave = (R*)(gw + G.rba);
    A.dwet = dwet;
    A.tacc = (double*)(gw + G.tacc);
    A.lpart = (double*)(gw + G.lpart);
    A.dLdrho = (const R*)r->dL_drho;
    A.NA = h->NA;
    A.NB = h->NB;
    A.NCc = h->NCc;
    A.N = N;
    A.omega = (R)(1.0 / p.tau[0]);
    for (int m = 0; m < q_of(p.lattice); ++m)
        A.srate[m] = (R)(p.mrt_s[0][m] / (p.lattice == LBM_D2Q9 ? mrt_norm<LAT_D2Q9>(m) : mrt_norm<LAT_D3Q19>(m)));
    A.eos_a = (R)p.eos_a[0];
    A.eos_b = (R)p.eos_b[0];
    A.eos_R = (R)p.eos_R[0];
    A.eos_T = (R)p.eos_T[0];
    A.alpha = (R)p.alpha[0];
    A.ginv = p.g[0][0] != 0.0 ? (R)(1.0 / p.g[0][0]) : (R)0;
    A.g = (R)p.g[0][0];
    A.A = (R)p.A[0];
    for (int d = 0; d < 3; ++d) A.body[d] = (R)p.body_accel[d];
    A.rho_min = (R)p.rho_min[0];
    A.rho_max = (R)p.rho_max[0];
    A.psi_cs = p.psi_kind[0] == LBM_PSI_CS;
    A.wet_drho = p.wet_mode[0] == LBM_WET_DRHO;
    A.obs = r->observable == LBM_OBS_SATURATION ? 0 : 1;
    A.rho_mid = (R)r->rho_mid;
    A.inv_delta = r->delta > 0.0 ? (R)(1.0 / r->delta) : (R)0;

    // fluid-node count for the saturation normaliser (from the stats reduction)
    {
        lbm_stats_t sx;
        const int rc = lbm_stats(h, &sx);
        if (rc == LBM_ERR_HIP) return rc;
        A.inv_npore = sx.n_fluid > 0 ? (R)(1.0 / (double)sx.n_fluid) : (R)0;
    }

    // forward run with a checkpoint at the start of every segment
    for (int s = 0; s < G.nseg; ++s) {
        e = hipMemcpyAsync(gw + G.ckpt + (size_t)s * G.state, state_ptr(h), G.state, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return LBM_ERR_HIP;
        const int len = (s + 1) * G.K <= r->nsteps ? G.K : r->nsteps - s * G.K;
        const int rc = lbm_step(h, len);
        if (rc) return rc;
    }
    e = hipMemsetAsync(dwet, 0, (size_t)N * 8, st);
    if (e == hipSuccess) e = hipMemsetAsync(gw + G.tacc, 0, (size_t)N * 8, st);
    if (e == hipSuccess) e = hipMemsetAsync(gw + G.lamA, 0, G.state, st);
    if (e == hipSuccess) e = hipMemsetAsync(gw + G.lamB, 0, G.state, st);
    if (e != hipSuccess) return LBM_ERR_HIP;

    // observable and adjoint seed at the final state
    R* lam_next = (R*)(gw + G.lamA);
    R* lam_cur = (R*)(gw + G.lamB);
    A.s = state_ptr(h);
    A.lam_out = lam_next;
    hipLaunchKernelGGL((k_adj_seed<LAT, R>), dim3(grid), dim3(blk), 0, st, A);
    hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(64), 0, st, A.lpart, grid, (double*)(gw + G.sums));

    // reverse sweep, segment by segment
    for (int s = G.nseg - 1; s >= 0; --s) {
        const int len = (s + 1) * G.K <= r->nsteps ? G.K : r->nsteps - s * G.K;
        char* seg = gw + G.seg;
        e = hipMemcpyAsync(seg, gw + G.ckpt + (size_t)s * G.state, G.state, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return LBM_ERR_HIP;
        for (int k = 0; k + 1 < len; ++k) {
            Buffers b{seg + (size_t)k * G.state, seg + (size_t)(k + 1) * G.state, nullptr, nullptr};
            if (run_step_buffers(h, b) != hipSuccess) return LBM_ERR_HIP;
        }
        for (int k = len - 1; k >= 0; --k) {
            A.s = seg + (size_t)k * G.state;
            A.lam_in = lam_next;
            A.lam_out = lam_cur;
            hipLaunchKernelGGL((k_adj_rho<LAT, R>), dim3(grid), dim3(blk), 0, st, A);
            hipLaunchKernelGGL((k_adj_psi<LAT, R>), dim3(grid), dim3(blk), 0, st, A);
            hipLaunchKernelGGL((k_adj_collide<LAT, R, COLL>), dim3(grid), dim3(blk), 0, st, A);
            hipLaunchKernelGGL((k_adj_psi_bar<LAT, R>), dim3(grid), dim3(blk), 0, st, A);
            hipLaunchKernelGGL((k_adj_stream<LAT, R>), dim3(grid), dim3(blk), 0, st, A);
            if (hipGetLastError() != hipSuccess) return LBM_ERR_HIP;
            R* t = lam_next;
            lam_next = lam_cur;
            lam_cur = t;
        }
    }
    {
        const int per = (N + kSumBlocks - 1) / kSumBlocks;
        hipLaunchKernelGGL(k_sum_partial, dim3(kSumBlocks), dim3(256), 0, st, (const double*)(gw + G.tacc),
                           N, per, (double*)(gw + G.tpart));
        hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(64), 0, st, (const double*)(gw + G.tpart), kSumBlocks,
                           (double*)(gw + G.sums) + 1);
    }
    // both sums use a fixed order, so the gradient is bitwise reproducible
    double sums[2];
    e = hipMemcpyAsync(sums, gw + G.sums, sizeof(sums), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return LBM_ERR_HIP;
    if (L_out) *L_out = sums[0];
    if (dT_out) *dT_out = sums[1];
    return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_grad_workspace_size(const lbm_handle* h, const lbm_grad_req* r, size_t* bytes_out) {
    const int rc = check_req(h, r);
    if (rc) return rc;
    if (!bytes_out) return LBM_ERR_ARG;
    *bytes_out = grad_layout(h, r).total;
    return LBM_OK;
}

int lbm_grad(lbm_handle* h, const lbm_grad_req* r, double* L_out, double* dwet_dev, double* dT_out) {
    int rc = check_req(h, r);
    if (rc) return rc;
    if (!dwet_dev || !r->ws) return LBM_ERR_ARG;
    if (r->ws_bytes < grad_layout(h, r).total) return LBM_ERR_SPACE;
    if (((uintptr_t)r->ws & 255u) != 0) return LBM_ERR_ARG;
    const bool d2 = h->p.lattice == LBM_D2Q9, mrt = h->p.collision == LBM_MRT;
    if (h->p.storage == LBM_STORE_F64) {
        if (d2) return mrt ? grad_impl<LAT_D2Q9, double, COLL_MRT>(h, r, L_out, dwet_dev, dT_out)
                           : grad_impl<LAT_D2Q9, double, COLL_BGK>(h, r, L_out, dwet_dev, dT_out);
        return mrt ? grad_impl<LAT_D3Q19, double, COLL_MRT>(h, r, L_out, dwet_dev, dT_out)
                   : grad_impl<LAT_D3Q19, double, COLL_BGK>(h, r, L_out, dwet_dev, dT_out);
    }
    if (d2) return mrt ? grad_impl<LAT_D2Q9, float, COLL_MRT>(h, r, L_out, dwet_dev, dT_out)
                       : grad_impl<LAT_D2Q9, float, COLL_BGK>(h, r, L_out, dwet_dev, dT_out);
    return mrt ? grad_impl<LAT_D3Q19, float, COLL_MRT>(h, r, L_out, dwet_dev, dT_out)
               : grad_impl<LAT_D3Q19, float, COLL_BGK>(h, r, L_out, dwet_dev, dT_out);
}

}  // extern "C"
