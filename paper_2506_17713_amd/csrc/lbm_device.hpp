// Device code of the fused multiphase lattice-Boltzmann step for gfx950.
//
// Layout in HBM (structure of arrays, x fastest):
//   populations  f[k][i][n]  (k component, i direction, n = (c*NB + b)*NA + a)
//   deviation storage adds rho*[k][n] in FP32
//   per-node neighbour word nbr[n]: bit 0 = node solid, bit i = node n - e_i solid
// Coordinates (a, b, c): 3-D lattices use (x, y, z); 2-D lattices use (x, -, y)
// with NB = 1, so a D2Q9 field has the same linear index y*nx + x.
//
// The step is pull-based: buffer A holds post-collision populations f*(t-1);
// one launch pulls f(x,t) = f*_i(x - e_i) (halfway bounce-back: f*_opp(i)(x)
// when x - e_i is solid), computes the moments, the virtual densities, the
// pseudopotential, the force, collides and stores f*(x,t) to buffer B at x.
//
// The force at x needs psi at x + e_j, which needs rho at x + e_j (one pull
// away) and, at a solid neighbour, the virtual density from rho at distance
// two.  A workgroup therefore owns a TA x TB column of the lattice and marches
// it along c: every plane is pulled once onto a rho ring of five planes (halo
// 2), turned into a psi/U ring of three planes (halo 1), and collided two
// planes behind the pull front.  No intermediate field touches HBM.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

namespace lbm {

enum { LAT_D2Q9 = 0, LAT_D3Q19 = 1 };
enum { COLL_BGK = 0, COLL_MRT = 1 };
enum { ST_F64 = 0, ST_F32 = 1, ST_F16 = 2, ST_BF16 = 3 };

// ---------------------------------------------------------------------------
// Compile-time iteration.
// ---------------------------------------------------------------------------
template <class F, int... Is>
__device__ __forceinline__ void sfor_impl(F&& f, std::integer_sequence<int, Is...>) {
    (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void sfor(F&& f) {
    sfor_impl(f, std::make_integer_sequence<int, N>{});
}

// ---------------------------------------------------------------------------
// Velocity sets.  Opposite directions are adjacent: opp(i) = i+1 for odd i.
// ---------------------------------------------------------------------------
template <int LAT> struct Lat;

template <> struct Lat<LAT_D3Q19> {
    static constexpr int Q = 19;
    static constexpr bool D3 = true;
    // physical components (x, y, z) = (a, b, c)
    static constexpr int ex[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    static constexpr int ey[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    static constexpr int ez[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    static constexpr int ea(int i) { return ex[i]; }
    static constexpr int eb(int i) { return ey[i]; }
    static constexpr int ec(int i) { return ez[i]; }
    static constexpr double w(int i) { return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0); }
};

template <> struct Lat<LAT_D2Q9> {
    static constexpr int Q = 9;
    static constexpr bool D3 = false;
    static constexpr int ex[9] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
    static constexpr int ey[9] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
    static constexpr int ez[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    // 2-D lattices march along y: (a, b, c) = (x, -, y)
    static constexpr int ea(int i) { return ex[i]; }
    static constexpr int eb(int) { return 0; }
    static constexpr int ec(int i) { return ey[i]; }
    static constexpr double w(int i) { return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0); }
};

__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// MRT moment rows: polynomials of the lattice velocity (Lallemand-Luo D2Q9,
// d'Humieres D3Q19), in the row order of lbm_params.mrt_s.
template <int LAT>
__host__ __device__ constexpr double mrt_coef(int m, int i) {
    using L = Lat<LAT>;
    const double x = L::ex[i], y = L::ey[i], z = L::ez[i];
    const double e2 = x * x + y * y + z * z;
    if constexpr (LAT == LAT_D2Q9) {
        switch (m) {
            case 0: return 1.0;
            case 1: return -4.0 + 3.0 * e2;
            case 2: return 4.0 - 10.5 * e2 + 4.5 * e2 * e2;
            case 3: return x;
            case 4: return (3.0 * e2 - 5.0) * x;
            case 5: return y;
            case 6: return (3.0 * e2 - 5.0) * y;
            case 7: return x * x - y * y;
            default: return x * y;
        }
    } else {
        switch (m) {
            case 0: return 1.0;
            case 1: return 19.0 * e2 - 30.0;
            case 2: return (21.0 * e2 * e2 - 53.0 * e2 + 24.0) / 2.0;
            case 3: return x;
            case 4: return (5.0 * e2 - 9.0) * x;
            case 5: return y;
            case 6: return (5.0 * e2 - 9.0) * y;
            case 7: return z;
            case 8: return (5.0 * e2 - 9.0) * z;
            case 9: return 3.0 * x * x - e2;
            case 10: return (3.0 * e2 - 5.0) * (3.0 * x * x - e2);
            case 11: return y * y - z * z;
            case 12: return (3.0 * e2 - 5.0) * (y * y - z * z);
            case 13: return x * y;
            case 14: return y * z;
            case 15: return x * z;
            case 16: return (y * y - z * z) * x;
            case 17: return (z * z - x * x) * y;
            default: return (x * x - y * y) * z;
        }
    }
}

// Squared norm of row m; the rows are orthogonal, so M^-1 = M^T diag(1/norm).
template <int LAT>
__host__ __device__ constexpr double mrt_norm(int m) {
    double s = 0.0;
    for (int i = 0; i < Lat<LAT>::Q; ++i) s += mrt_coef<LAT>(m, i) * mrt_coef<LAT>(m, i);
    return s;
}

// ---------------------------------------------------------------------------
// Population storage formats.
// ---------------------------------------------------------------------------
template <int ST> struct Store;
template <> struct Store<ST_F64> {
    using S = double;
    using R = double;
    static constexpr bool DEV = false;
};
template <> struct Store<ST_F32> {
    using S = float;
    using R = float;
    static constexpr bool DEV = false;
};
template <> struct Store<ST_F16> {
    using S = _Float16;
    using R = float;
    static constexpr bool DEV = true;
    static __device__ __forceinline__ float load(S v) { return (float)v; }
    static __device__ __forceinline__ S cvt(float v) { return (_Float16)v; }  // RNE
};
template <> struct Store<ST_BF16> {
    using S = uint16_t;
    using R = float;
    static constexpr bool DEV = true;
    static __device__ __forceinline__ float load(S v) { return __uint_as_float((uint32_t)v << 16); }
    // round to nearest, ties to even; NaN stays NaN
    static __device__ __forceinline__ S cvt(float v) {
        uint32_t u = __float_as_uint(v);
        if ((u & 0x7fffffffu) > 0x7f800000u) return (S)((u >> 16) | 0x40u);
        u += 0x7fffu + ((u >> 16) & 1u);
        return (S)(u >> 16);
    }
};

// ---------------------------------------------------------------------------
// Kernel arguments (by value).
// ---------------------------------------------------------------------------
template <class R>
struct StepArgs {
    const void* fin;       // populations at t-1 (post-collision)
    void* fout;            // populations written by this step
    const float* rin;      // deviation storage: rho* at t-1 [NC][N]
    float* rout;           // deviation storage: rho* written [NC][N]
    const uint32_t* nbr;   // neighbour words [N]
    const R* wet;          // wetting parameter [NC][N] (read at solid nodes)
    R* mom_rho;            // moments output [N]
    R* mom_u;              // moments output [3][N]
    int mom_comp;          // component, or -1 for the mixture
    int NA, NB, NC_;       // extents along a, b, c
    int tiles_a, tiles_b, chunk;
    int N;                 // nodes
    int psi_cs[2];         // 1: Carnahan-Starling pseudopotential, 0: psi = rho
    int wet_drho[2];       // 1: rho_ave - drho, 0: phi * rho_ave
    int common_u;          // two components: common equilibrium velocity
    int has_zc;            // any A_kk != 0
    R omega[2];            // 1/tau
    R srate[2][19];        // MRT: s_m / |row m|^2
    R eos_a[2], eos_b[2], eos_RT[2], alpha[2], ginv[2];  // ginv = 1/g_kk
    R A[2];
    R g[2][2];
    R body[3];
    R rho_min[2], rho_max[2];
};

__device__ __forceinline__ int wrap_near(int v, int n) {
    // v in [-n, 2n)
    return v < 0 ? v + n : (v >= n ? v - n : v);
}
__device__ __forceinline__ int wrap_any(int v, int n) {
    int r = v % n;
    return r < 0 ? r + n : r;
}

// ---------------------------------------------------------------------------
// Pull of all directions of one node (all components).
// ---------------------------------------------------------------------------
template <int LAT, int ST, int NC>
__device__ __forceinline__ void pull_node(const StepArgs<typename Store<ST>::R>& P, int n, int a,
                                          int b, int c, uint32_t word,
                                          typename Store<ST>::R (&f)[NC][Lat<LAT>::Q]) {
    using L = Lat<LAT>;
    using SS = Store<ST>;
    using S = typename SS::S;
    using R = typename SS::R;
    constexpr int Q = L::Q;
    const int NA = P.NA, NB = P.NB, NCc = P.NC_;
    const int plane = NA * NB;
    // index deltas of the neighbour at -1, 0, +1 along each axis (periodic)
    const int dA[3] = {a == 0 ? NA - 1 : -1, 0, a == NA - 1 ? 1 - NA : 1};
    const int dB[3] = {b == 0 ? (NB - 1) * NA : -NA, 0, b == NB - 1 ? (1 - NB) * NA : NA};
    const int dC[3] = {c == 0 ? (NCc - 1) * plane : -plane, 0, c == NCc - 1 ? (1 - NCc) * plane : plane};
    const S* fin = reinterpret_cast<const S*>(P.fin);
    const size_t N = (size_t)P.N;
    // streaming loads do not depend on the neighbour word, so they issue
    // together with it; a source that is solid holds no population and its
    // value is replaced by the bounced one below
    S v[NC][Q];
    float rs[NC][Q];
    sfor<Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        const int src = n + dA[1 - L::ea(i)] + dB[1 - L::eb(i)] + dC[1 - L::ec(i)];
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            v[k][i] = fin[(size_t)(k * Q + i) * N + src];
            if constexpr (SS::DEV) rs[k][i] = P.rin[(size_t)k * N + src];
        }
    });
    if (word & ~1u) {
        // halfway bounce-back: f_i(x) = f*_opp(i)(x) when x - e_i is solid
        sfor<Q - 1>([&](auto I) {
            constexpr int i = decltype(I)::value + 1;
            constexpr int o = opp(i);
            if ((word >> i) & 1u) {
#pragma unroll
                for (int k = 0; k < NC; ++k) {
                    v[k][i] = fin[(size_t)(k * Q + o) * N + n];
                    if constexpr (SS::DEV) rs[k][i] = P.rin[(size_t)k * N + n];
                }
            }
        });
    }
    sfor<Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            if constexpr (SS::DEV) f[k][i] = (float)L::w(i) * rs[k][i] * (1.0f + SS::load(v[k][i]));
            else f[k][i] = (R)v[k][i];
        }
    });
}

// ---------------------------------------------------------------------------
// Pseudopotential (Eq. 12): psi = sqrt(2 (alpha p_CS - c_s^2 rho) / g_kk),
// U = alpha p_CS - c_s^2 rho; psi = rho for the density pseudopotential.
// ---------------------------------------------------------------------------
template <class R>
__device__ __forceinline__ void psi_of(const StepArgs<R>& P, int k, R rho, R& psi, R& U) {
    if (P.psi_cs[k]) {
        const R eta = P.eos_b[k] * rho * (R)0.25;
        const R om = (R)1 - eta;
        const R p = rho * P.eos_RT[k] * ((R)1 + eta + eta * eta - eta * eta * eta) / (om * om * om) -
                    P.eos_a[k] * rho * rho;
        const R u = P.alpha[k] * p - rho * (R)(1.0 / 3.0);
        R arg = (R)2 * u * P.ginv[k];
        arg = arg > (R)0 ? arg : (R)0;
        psi = sqrt(arg);
        U = u;
    } else {
        psi = rho;
        U = (R)0;
    }
}

// ---------------------------------------------------------------------------
// The fused step (MOM = false) or the moment evaluation (MOM = true).
// ---------------------------------------------------------------------------
#ifndef LBM_WAVES_PER_EU
#define LBM_WAVES_PER_EU 1
#endif
template <int LAT, int NC, int ST, int COLL, bool MOM, int TA, int TB, bool CARRY>
__global__ void __launch_bounds__(TA* TB) __attribute__((amdgpu_waves_per_eu(LBM_WAVES_PER_EU)))
    k_step(StepArgs<typename Store<ST>::R> P) {
    using L = Lat<LAT>;
    using SS = Store<ST>;
    using S = typename SS::S;
    using R = typename SS::R;
    constexpr int Q = L::Q;
    constexpr bool D3 = L::D3;
    constexpr int NT = TA * TB;
    constexpr int H2B = D3 ? 2 : 0;  // rho halo along b
    constexpr int H1B = D3 ? 1 : 0;  // psi halo along b
    constexpr int RWA = TA + 4, RWB = TB + 2 * H2B, RP = RWA * RWB;
    constexpr int PWA = TA + 2, PWB = TB + 2 * H1B, PP = PWA * PWB;

    __shared__ R s_rho[5][NC][RP];  // rho of fluid nodes, -1 at solid nodes
    __shared__ R s_psi[3][NC][PP];
    __shared__ R s_U[3][NC][PP];

    const int tid = threadIdx.x;
    const int NA = P.NA, NB = P.NB, NCc = P.NC_;
    const size_t N = (size_t)P.N;

    // XCD-aware tile order: consecutive tiles land on the same XCD (the
    // hardware deals workgroups round-robin over 8 XCDs).
    const int nblk = gridDim.x, bid = blockIdx.x;
    const int per = nblk >> 3, rem = nblk & 7, xcd = bid & 7;
    const int tile = xcd * per + (xcd < rem ? xcd : rem) + (bid >> 3);
    const int ta = tile % P.tiles_a;
    const int tb = (tile / P.tiles_a) % P.tiles_b;
    const int ch = tile / (P.tiles_a * P.tiles_b);
    const int a0 = ta * TA, b0 = tb * TB;
    const int c0 = ch * P.chunk;
    const int c1 = (c0 + P.chunk < NCc) ? c0 + P.chunk : NCc;
    const bool smallA = NA < RWA, smallB = NB < RWB;

    auto wrap_c = [&](int cp) { return NCc < 5 ? wrap_any(cp, NCc) : wrap_near(cp, NCc); };
    auto rho_sum = [&](const R(&f)[NC][Q], int k) {
        R r = f[k][0];
        sfor<(Q - 1) / 2>([&](auto PI) {
            constexpr int i = 2 * decltype(PI)::value + 1;
            r += f[k][i] + f[k][i + 1];
        });
        return r;
    };

    // ---- phase 1: pull a plane with halo 2, store rho (solid: -1) ---------
    // Each thread pulls its own node (kept in registers until its collision
    // two planes later when CARRY) and HPT halo positions.  A halo-2 position
    // (outside the psi halo) only feeds virtual densities and is pulled only
    // when it has a solid neighbour.  The neighbour words of the next plane
    // are fetched one plane ahead so that no pull waits for them.
    const int la_own = tid % TA, lb_own = tid / TA;
    const int own_idx = (lb_own + H2B) * RWA + la_own + 2;
    constexpr int HALO = RP - NT;
    constexpr int HPT = (HALO + NT - 1) / NT;
    int own_a = a0 + la_own, own_b = b0 + lb_own;
    own_a = smallA ? wrap_any(own_a, NA) : wrap_near(own_a, NA);
    own_b = D3 ? (smallB ? wrap_any(own_b, NB) : wrap_near(own_b, NB)) : 0;
    int h_idx[HPT], h_a[HPT], h_b[HPT];
    bool h_on[HPT], h_outer[HPT];
#pragma unroll
    for (int j = 0; j < HPT; ++j) {
        constexpr int TOP = H2B * RWA;
        const int h = tid + j * NT;
        h_on[j] = h < HALO;
        const int hh = h_on[j] ? h : 0;
        int ra, rb;
        if (hh < TOP) {
            rb = hh / RWA;
            ra = hh % RWA;
        } else if (hh < 2 * TOP) {
            rb = TB + H2B + (hh - TOP) / RWA;
            ra = (hh - TOP) % RWA;
        } else {
            const int h3 = hh - 2 * TOP;
            rb = H2B + h3 / 4;
            const int c4 = h3 % 4;
            ra = c4 < 2 ? c4 : TA + c4;
        }
        h_outer[j] = ra == 0 || ra == RWA - 1 || (D3 && (rb == 0 || rb == RWB - 1));
        h_idx[j] = rb * RWA + ra;
        int ha = a0 + ra - 2, hb = b0 + rb - H2B;
        h_a[j] = smallA ? wrap_any(ha, NA) : wrap_near(ha, NA);
        h_b[j] = D3 ? (smallB ? wrap_any(hb, NB) : wrap_near(hb, NB)) : 0;
    }
    uint32_t w_own = 0, w_halo[HPT];
    auto fetch_words = [&](int cp) {
        const int c = wrap_c(cp);
        w_own = P.nbr[(c * NB + own_b) * NA + own_a];
#pragma unroll
        for (int j = 0; j < HPT; ++j) w_halo[j] = h_on[j] ? P.nbr[(c * NB + h_b[j]) * NA + h_a[j]] : 0u;
    };
    auto fill_rho = [&](int cp, R(&fo)[NC][Q]) {
        const int slot = (cp - c0 + 5) % 5;
        const int c = wrap_c(cp);
        const uint32_t wo = w_own;
        uint32_t wh[HPT];
#pragma unroll
        for (int j = 0; j < HPT; ++j) wh[j] = w_halo[j];
        fetch_words(cp + 1);
        {
            const int n = (c * NB + own_b) * NA + own_a;
            pull_node<LAT, ST, NC>(P, n, own_a, own_b, c, wo, fo);
            if (wo & 1u) {
#pragma unroll
                for (int k = 0; k < NC; ++k) s_rho[slot][k][own_idx] = (R)-1;
            } else {
#pragma unroll
                for (int k = 0; k < NC; ++k) s_rho[slot][k][own_idx] = rho_sum(fo, k);
            }
        }
#pragma unroll
        for (int j = 0; j < HPT; ++j) {
            if (!h_on[j]) continue;
            if (wh[j] & 1u) {
#pragma unroll
                for (int k = 0; k < NC; ++k) s_rho[slot][k][h_idx[j]] = (R)-1;
            } else if (h_outer[j] && wh[j] == 0u) {
#pragma unroll
                for (int k = 0; k < NC; ++k) s_rho[slot][k][h_idx[j]] = (R)0;  // never read
            } else {
                R f[NC][Q];
                pull_node<LAT, ST, NC>(P, (c * NB + h_b[j]) * NA + h_a[j], h_a[j], h_b[j], c, wh[j], f);
#pragma unroll
                for (int k = 0; k < NC; ++k) s_rho[slot][k][h_idx[j]] = rho_sum(f, k);
            }
        }
    };

    // ---- phase 2: psi and U of a plane with halo 1 (Eq. 12, Eq. 17) -------
    auto fill_psi = [&](int cp) {
        const int pslot = (cp - c0 + 3) % 3;
        const int rs0 = (cp - c0 + 5) % 5;
        for (int idx = tid; idx < PP; idx += NT) {
            const int pa = idx % PWA, pb = idx / PWA;
            const int ra = pa + 1, rb = pb + (H2B - H1B);
            const R r0 = s_rho[rs0][0][rb * RWA + ra];
            if (r0 >= (R)0) {
#pragma unroll
                for (int k = 0; k < NC; ++k) {
                    R ps, u;
                    psi_of(P, k, s_rho[rs0][k][rb * RWA + ra], ps, u);
                    s_psi[pslot][k][idx] = ps;
                    s_U[pslot][k][idx] = u;
                }
            } else {
                // solid: weighted average of fluid-neighbour densities
                R num[NC], den = 0;
#pragma unroll
                for (int k = 0; k < NC; ++k) num[k] = 0;
                sfor<Q - 1>([&](auto I) {
                    constexpr int i = decltype(I)::value + 1;
                    const int sl = (cp + L::ec(i) - c0 + 5) % 5;
                    const int off = (rb + L::eb(i)) * RWA + ra + L::ea(i);
                    const R v0 = s_rho[sl][0][off];
                    if (v0 >= (R)0) {
                        den += (R)L::w(i);
#pragma unroll
                        for (int k = 0; k < NC; ++k) num[k] += (R)L::w(i) * s_rho[sl][k][off];
                    }
                });
                if (den > (R)0) {
                    const int c = NCc < 5 ? wrap_any(cp, NCc) : wrap_near(cp, NCc);
                    int a = a0 + pa - 1, b = b0 + pb - H1B;
                    a = smallA ? wrap_any(a, NA) : wrap_near(a, NA);
                    b = D3 ? (smallB ? wrap_any(b, NB) : wrap_near(b, NB)) : 0;
                    const int n = (c * NB + b) * NA + a;
#pragma unroll
                    for (int k = 0; k < NC; ++k) {
                        const R rave = num[k] / den;
                        const R prm = P.wet[(size_t)k * N + n];
                        R rsv = P.wet_drho[k] ? rave - prm : prm * rave;
                        rsv = rsv < P.rho_min[k] ? P.rho_min[k] : rsv;
                        rsv = rsv > P.rho_max[k] ? P.rho_max[k] : rsv;
                        R ps, u;
                        psi_of(P, k, rsv, ps, u);
                        s_psi[pslot][k][idx] = ps;
                        s_U[pslot][k][idx] = u;
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < NC; ++k) {
                        s_psi[pslot][k][idx] = 0;
                        s_U[pslot][k][idx] = 0;
                    }
                }
            }
        }
    };

    // ---- phase 3: force, collision + EDM, store (or moments) --------------
    auto collide_f = [&](int c, const R(&f)[NC][Q], bool pulled) {
        const int la = la_own, lb = lb_own;
        const int a = a0 + la, b = b0 + lb;
        if (a >= NA || b >= NB) return;
        const int n = (c * NB + b) * NA + a;
        const uint32_t word = P.nbr[n];
        if (word & 1u) {
            if constexpr (MOM) {
                if (P.mom_rho) P.mom_rho[n] = 0;
                if (P.mom_u) {
                    P.mom_u[n] = 0;
                    P.mom_u[N + n] = 0;
                    P.mom_u[2 * N + n] = 0;
                }
            }
            return;
        }
        (void)pulled;
        // moments (Eq. 4); the momentum is summed over differences of opposite
        // populations, which are exact in floating point when the two are
        // within a factor of two of each other (Sterbenz)
        R rho[NC], j[NC][3];
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            R r = f[k][0], jx = 0, jy = 0, jz = 0;
            sfor<(Q - 1) / 2>([&](auto PI) {
                constexpr int i = 2 * decltype(PI)::value + 1;  // e_{i+1} = -e_i
                r += f[k][i] + f[k][i + 1];
                const R d = f[k][i] - f[k][i + 1];
                if constexpr (L::ex[i] != 0) jx += L::ex[i] > 0 ? d : -d;
                if constexpr (L::ey[i] != 0) jy += L::ey[i] > 0 ? d : -d;
                if constexpr (L::ez[i] != 0) jz += L::ez[i] > 0 ? d : -d;
            });
            rho[k] = r;
            j[k][0] = jx;
            j[k][1] = jy;
            j[k][2] = jz;
        }
        // interaction force (Eq. 13) with G_i = w_i / c_s^2
        const int sc = (c - c0 + 3) % 3;
        const int pc = (lb + H1B) * PWA + la + 1;
        R F[NC][3];
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            // sum_i G_i psi(x + e_i) e_i taken as differences across opposite
            // neighbours, psi(x + e_i) - psi(x - e_i)
            R sx = 0, sy = 0, sz = 0, zx = 0, zy = 0, zz = 0;
            sfor<(Q - 1) / 2>([&](auto PI) {
                constexpr int i = 2 * decltype(PI)::value + 1;
                constexpr R G = (R)(3.0 * L::w(i));
                const int slp = (c + L::ec(i) - c0 + 3) % 3;
                const int slm = (c - L::ec(i) - c0 + 3) % 3;
                const int offp = pc + L::eb(i) * PWA + L::ea(i);
                const int offm = pc - L::eb(i) * PWA - L::ea(i);
                R s = 0;
#pragma unroll
                for (int kk = 0; kk < NC; ++kk)
                    s += P.g[k][kk] * (s_psi[slp][kk][offp] - s_psi[slm][kk][offm]);
                s *= G;
                if constexpr (L::ex[i] != 0) sx += L::ex[i] > 0 ? s : -s;
                if constexpr (L::ey[i] != 0) sy += L::ey[i] > 0 ? s : -s;
                if constexpr (L::ez[i] != 0) sz += L::ez[i] > 0 ? s : -s;
                if (P.has_zc) {
                    const R uu = G * (s_U[slp][k][offp] - s_U[slm][k][offm]);
                    if constexpr (L::ex[i] != 0) zx += L::ex[i] > 0 ? uu : -uu;
                    if constexpr (L::ey[i] != 0) zy += L::ey[i] > 0 ? uu : -uu;
                    if constexpr (L::ez[i] != 0) zz += L::ez[i] > 0 ? uu : -uu;
                }
            });
            const R psik = s_psi[sc][k][pc];
            const R Ak = P.A[k], Bk = (R)1 - P.A[k];
            F[k][0] = -Ak * zx - Bk * psik * sx + rho[k] * P.body[0];
            F[k][1] = -Ak * zy - Bk * psik * sy + rho[k] * P.body[1];
            F[k][2] = -Ak * zz - Bk * psik * sz + rho[k] * P.body[2];
        }

        if constexpr (MOM) {
            // Eq. 6: u = (j + F/2) / rho, per component or for the mixture
            R rr = 0, mx = 0, my = 0, mz = 0;
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                if (P.mom_comp < 0 || P.mom_comp == k) {
                    rr += rho[k];
                    mx += j[k][0] + (R)0.5 * F[k][0];
                    my += j[k][1] + (R)0.5 * F[k][1];
                    mz += j[k][2] + (R)0.5 * F[k][2];
                }
            }
            if (P.mom_rho) P.mom_rho[n] = rr;
            if (P.mom_u) {
                const R inv = (R)1 / rr;
                P.mom_u[n] = mx * inv;
                P.mom_u[N + n] = my * inv;
                P.mom_u[2 * N + n] = mz * inv;
            }
        } else {
            // equilibrium velocity: j/rho, or the common u' for two components
            R ueq[NC][3];
            if (NC > 1 && P.common_u) {
                R nx_ = 0, ny_ = 0, nz_ = 0, d = 0;
#pragma unroll
                for (int k = 0; k < NC; ++k) {
                    nx_ += j[k][0] * P.omega[k];
                    ny_ += j[k][1] * P.omega[k];
                    nz_ += j[k][2] * P.omega[k];
                    d += rho[k] * P.omega[k];
                }
                const R inv = (R)1 / d;
#pragma unroll
                for (int k = 0; k < NC; ++k) {
                    ueq[k][0] = nx_ * inv;
                    ueq[k][1] = ny_ * inv;
                    ueq[k][2] = nz_ * inv;
                }
            } else {
#pragma unroll
                for (int k = 0; k < NC; ++k) {
                    const R inv = (R)1 / rho[k];
                    ueq[k][0] = j[k][0] * inv;
                    ueq[k][1] = j[k][1] * inv;
                    ueq[k][2] = j[k][2] * inv;
                }
            }
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                const R r = rho[k];
                const R invr = (R)1 / r;
                const R ux = ueq[k][0], uy = ueq[k][1], uz = ueq[k][2];
                // velocity increment of the exact-difference method, du = F / rho
                const R dx = F[k][0] * invr, dy = F[k][1] * invr, dz = F[k][2] * invr;
                const R usq = (R)1.5 * (ux * ux + uy * uy + uz * uz);
                const R dsq = (R)1.5 * ((R)2 * (ux * dx + uy * dy + uz * dz) + dx * dx + dy * dy + dz * dz);
                R feq[Q], dF[Q];
                sfor<Q>([&](auto I) {
                    constexpr int i = decltype(I)::value;
                    constexpr R ex = L::ex[i], ey = L::ey[i], ez = L::ez[i];
                    const R wr = (R)L::w(i) * r;
                    const R eu = ex * ux + ey * uy + ez * uz;
                    const R ed = ex * dx + ey * dy + ez * dz;
                    feq[i] = wr * ((R)1 + (R)3 * eu + (R)4.5 * eu * eu - usq);
                    // Eq. 5: f^eq(rho, u + du) - f^eq(rho, u), expanded so that no
                    // two O(w rho) numbers are subtracted
                    dF[i] = wr * (ed * ((R)3 + (R)4.5 * ((R)2 * eu + ed)) - dsq);
                });
                R fo[Q];
                if constexpr (COLL == COLL_BGK) {
                    const R om = P.omega[k];
#pragma unroll
                    for (int i = 0; i < Q; ++i) fo[i] = f[k][i] - om * (f[k][i] - feq[i]) + dF[i];
                } else {
                    R d[Q], m[Q];
#pragma unroll
                    for (int i = 0; i < Q; ++i) d[i] = f[k][i] - feq[i];
                    sfor<Q>([&](auto M) {
                        constexpr int mm = decltype(M)::value;
                        R s = 0;
                        sfor<Q>([&](auto I) {
                            constexpr int i = decltype(I)::value;
                            constexpr double cf = mrt_coef<LAT>(mm, i);
                            if constexpr (cf == 1.0) s += d[i];
                            else if constexpr (cf == -1.0) s -= d[i];
                            else if constexpr (cf != 0.0) s += (R)cf * d[i];
                        });
                        m[mm] = s * P.srate[k][mm];
                    });
                    sfor<Q>([&](auto I) {
                        constexpr int i = decltype(I)::value;
                        R s = 0;
                        sfor<Q>([&](auto M) {
                            constexpr int mm = decltype(M)::value;
                            constexpr double cf = mrt_coef<LAT>(mm, i);
                            if constexpr (cf == 1.0) s += m[mm];
                            else if constexpr (cf == -1.0) s -= m[mm];
                            else if constexpr (cf != 0.0) s += (R)cf * m[mm];
                        });
                        fo[i] = f[k][i] - s + dF[i];
                    });
                }
                // collision and forcing conserve mass exactly; the rest population
                // takes the remainder so that sum_i f*_i = rho holds to rounding
                {
                    R m = 0;
                    sfor<(Q - 1) / 2>([&](auto PI) {
                        constexpr int i = 2 * decltype(PI)::value + 1;
                        m += fo[i] + fo[i + 1];
                    });
                    fo[0] = r - m;
                }
                // store
                if constexpr (SS::DEV) {
                    float* ro = P.rout;
                    ro[(size_t)k * N + n] = r;
                    const float ir = 1.0f / r;
                    S* out = reinterpret_cast<S*>(P.fout);
                    sfor<Q>([&](auto I) {
                        constexpr int i = decltype(I)::value;
                        constexpr float iw = (float)(1.0 / L::w(i));
                        out[(size_t)(k * Q + i) * N + n] = SS::cvt(fo[i] * (iw * ir) - 1.0f);
                    });
                } else {
                    S* out = reinterpret_cast<S*>(P.fout);
#pragma unroll
                    for (int i = 0; i < Q; ++i) out[(size_t)(k * Q + i) * N + n] = fo[i];
                }
            }
        }
    };

    // ---- pipeline along c ---------------------------------------------------
    // Iteration it pulls plane it+2, evaluates psi of plane it+1 and collides
    // plane it; the first four iterations only fill the rings.  One loop body
    // keeps the code small enough for the instruction cache.
    R fc0[NC][Q], fc1[NC][Q], fc2[NC][Q];
    fetch_words(c0 - 2);
#pragma nounroll
    for (int it = c0 - 4; it < c1; ++it) {
        fill_rho(it + 2, fc2);
        __syncthreads();
        if (it + 1 >= c0 - 1) fill_psi(it + 1);
        __syncthreads();
        if (it >= c0) {
            if constexpr (CARRY) {
                collide_f(it, fc0, false);
            } else {
                // re-pull the own node (L2-resident since its ring pull)
                const int a = a0 + la_own, b = b0 + lb_own;
                if (a < NA && b < NB) {
                    const int n = (it * NB + b) * NA + a;
                    const uint32_t word = P.nbr[n];
                    if (!(word & 1u)) pull_node<LAT, ST, NC>(P, n, a, b, it, word, fc0);
                    collide_f(it, fc0, true);
                }
            }
        }
        if constexpr (CARRY) {
#pragma unroll
            for (int k = 0; k < NC; ++k)
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    fc0[k][i] = fc1[k][i];
                    fc1[k][i] = fc2[k][i];
                }
        }
    }
}

// ---------------------------------------------------------------------------
// Initialisation kernels.
// ---------------------------------------------------------------------------
// Neighbour words: bit 0 = node solid, bit i = node n - e_i solid.
template <int LAT>
__global__ void k_nbr_words(const uint8_t* __restrict__ mask, uint32_t* __restrict__ nbr, int NA,
                            int NB, int NCc) {
    using L = Lat<LAT>;
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    const int N = NA * NB * NCc;
    if (n >= N) return;
    const int a = n % NA, b = (n / NA) % NB, c = n / (NA * NB);
    uint32_t w = mask[n] ? 1u : 0u;
    sfor<L::Q - 1>([&](auto I) {
        constexpr int i = decltype(I)::value + 1;
        const int aa = wrap_any(a - L::ea(i), NA);
        const int bb = wrap_any(b - L::eb(i), NB);
        const int cc = wrap_any(c - L::ec(i), NCc);
        if (mask[(cc * NB + bb) * NA + aa]) w |= 1u << i;
    });
    nbr[n] = w;
}

// Populations such that the first pull gives f = f^eq(rho0, u0) at every
// fluid node: f*_i(y) = f^eq_i(y + e_i) when y + e_i is fluid, else the
// population bounced back into y, f^eq_opp(i)(y).
template <int LAT, int NC, int ST>
__global__ void k_init(const typename Store<ST>::R* __restrict__ rho0,
                       const typename Store<ST>::R* __restrict__ u0, const uint32_t* __restrict__ nbr,
                       void* fout, float* rout, int NA, int NB, int NCc) {
    using L = Lat<LAT>;
    using SS = Store<ST>;
    using S = typename SS::S;
    using R = typename SS::R;
    constexpr int Q = L::Q;
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    const int N = NA * NB * NCc;
    if (n >= N) return;
    const uint32_t word = nbr[n];
    S* out = reinterpret_cast<S*>(fout);
    const int a = n % NA, b = (n / NA) % NB, c = n / (NA * NB);
    auto feq = [&](int k, int m, int i, int ex, int ey, int ez, double wi) -> R {
        const R r = rho0[(size_t)k * N + m];
        const R ux = u0 ? u0[m] : (R)0, uy = u0 ? u0[(size_t)N + m] : (R)0, uz = u0 ? u0[2 * (size_t)N + m] : (R)0;
        const R eu = ex * ux + ey * uy + ez * uz;
        return (R)wi * r * ((R)1 + (R)3 * eu + (R)4.5 * eu * eu - (R)1.5 * (ux * ux + uy * uy + uz * uz));
    };
    for (int k = 0; k < NC; ++k) {
        const R r0 = rho0[(size_t)k * N + n];
        if constexpr (SS::DEV) rout[(size_t)k * N + n] = (word & 1u) ? 0.0f : (float)r0;
        sfor<Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            constexpr int o = opp(i);
            R v = 0;
            if (!(word & 1u)) {
                if ((word >> o) & 1u && i != 0) {
                    v = feq(k, n, o, L::ex[o], L::ey[o], L::ez[o], L::w(o));
                } else {
                    const int aa = wrap_any(a + L::ea(i), NA);
                    const int bb = wrap_any(b + L::eb(i), NB);
                    const int cc = wrap_any(c + L::ec(i), NCc);
                    const int m = (cc * NB + bb) * NA + aa;
                    v = feq(k, m, i, L::ex[i], L::ey[i], L::ez[i], L::w(i));
                }
            }
            if constexpr (SS::DEV) {
                const float h = (word & 1u) ? 0.0f : (float)v / ((float)L::w(i) * (float)r0) - 1.0f;
                out[(size_t)(k * Q + i) * N + n] = SS::cvt(h);
            } else {
                out[(size_t)(k * Q + i) * N + n] = (S)v;
            }
        });
    }
}

}  // namespace lbm
