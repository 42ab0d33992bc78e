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
enum { COLL_BGK = 0, COLL_MRT = 1, COLL_CLBM = 2 };
enum { ST_F64 = 0, ST_F32 = 1, ST_F16 = 2, ST_BF16 = 3, ST_F32D = 4 };

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

// Row m is even (same coefficient on e_i and -e_i) or odd (opposite sign).
template <int LAT>
__host__ __device__ constexpr bool mrt_even(int m) {
    for (int i = 1; i < Lat<LAT>::Q; ++i)
        if (mrt_coef<LAT>(m, i) != mrt_coef<LAT>(m, opp(i))) return false;
    return true;
}
// Row m is a momentum component (e_x, e_y or e_z).
template <int LAT>
__host__ __device__ constexpr bool mrt_momentum(int m) {
    using L = Lat<LAT>;
    bool isx = true, isy = true, isz = LAT == LAT_D3Q19;
    for (int i = 0; i < L::Q; ++i) {
        isx = isx && mrt_coef<LAT>(m, i) == L::ex[i];
        isy = isy && mrt_coef<LAT>(m, i) == L::ey[i];
        isz = isz && mrt_coef<LAT>(m, i) == L::ez[i];
    }
    return isx || isy || isz;
}

// D3Q19 MRT in pair form.  Pair p holds directions 2p+1 and 2p+2 (opposite);
// dp = d_i + d_{i+1}, dm = d_i - d_{i+1} of d = f - f^eq, d0 the rest entry.
// Applies m = diag(s) M d (rows of mrt_coef, s already divided by |row|^2)
// and returns M^T m as E (even rows) and O (odd rows): (M^T m)_{2p+1} = E_p +
// O_p, (M^T m)_{2p+2} = E_p - O_p.  Rows 0 (density) and, unless JROWS, 3, 5,
// 7 (momentum) are left out.  The row sums are factored over the shared
// sub-sums of each |e|^2 class: the products are those of mrt_coef, in fewer
// operations (pinned to the full matrix product by the parity tests).
template <class R, bool JROWS>
__host__ __device__ __forceinline__ void mrt_pairs_d3q19(const R (&dp)[9], const R (&dm)[9], R d0,
                                                         const R (&s)[19], R (&E)[9], R (&O)[9]) {
    // even rows: 1, 2 (energy), 9-12 (normal stress), 13-15 (shear)
    const R A = dp[0] + dp[1] + dp[2];
    const R C = dp[3] + dp[4], D = dp[5] + dp[6], G = dp[7] + dp[8];
    const R B = C + D + G;
    const R m1 = ((R)-30 * d0 - (R)11 * A + (R)8 * B) * s[1];
    const R m2 = ((R)12 * d0 - (R)4 * A + B) * s[2];
    const R Y = (R)2 * dp[0] - (dp[1] + dp[2]);
    const R X = (C + D) - (R)2 * G;
    const R m9 = (Y + X) * s[9];
    const R m10 = (X - (R)2 * Y) * s[10];
    const R Z = dp[1] - dp[2], W = C - D;
    const R m11 = (Z + W) * s[11];
    const R m12 = (W - (R)2 * Z) * s[12];
    const R m13 = (dp[3] - dp[4]) * s[13];
    const R m14 = (dp[7] - dp[8]) * s[14];
    const R m15 = (dp[5] - dp[6]) * s[15];
    // odd rows: 3, 5, 7 (momentum), 4, 6, 8 (energy flux), 16-18
    const R Px = dm[3] + dm[4], Qx = dm[5] + dm[6];
    const R Ry = dm[3] - dm[4], Sy = dm[7] + dm[8];
    const R Tz = dm[5] - dm[6], Uz = dm[7] - dm[8];
    const R m4 = ((R)-4 * dm[0] + Px + Qx) * s[4];
    const R m6 = ((R)-4 * dm[1] + Ry + Sy) * s[6];
    const R m8 = ((R)-4 * dm[2] + Tz + Uz) * s[8];
    const R m16 = (Px - Qx) * s[16];
    const R m17 = (Sy - Ry) * s[17];
    const R m18 = (Tz - Uz) * s[18];
    R m3 = 0, m5 = 0, m7 = 0;
    if constexpr (JROWS) {
        m3 = (dm[0] + Px + Qx) * s[3];
        m5 = (dm[1] + Ry + Sy) * s[5];
        m7 = (dm[2] + Tz + Uz) * s[7];
    }
    // back: even part
    const R Ea = (R)-11 * m1 - (R)4 * m2, Ed = (R)8 * m1 + m2;
    const R K = m9 + m10, L2 = m11 + m12;
    E[0] = Ea + (R)2 * m9 - (R)4 * m10;
    const R v1 = (R)2 * m10 - m9, h1 = m11 - (R)2 * m12;
    E[1] = Ea + v1 + h1;
    E[2] = Ea + v1 - h1;
    const R b34 = Ed + K + L2, b56 = Ed + K - L2, b78 = Ed - (R)2 * K;
    E[3] = b34 + m13;
    E[4] = b34 - m13;
    E[5] = b56 + m15;
    E[6] = b56 - m15;
    E[7] = b78 + m14;
    E[8] = b78 - m14;
    // back: odd part
    const R X4 = m3 + m4, Y6 = m5 + m6, Z8 = m7 + m8;
    O[0] = m3 - (R)4 * m4;
    O[1] = m5 - (R)4 * m6;
    O[2] = m7 - (R)4 * m8;
    O[3] = X4 + Y6 + (m16 - m17);
    O[4] = X4 - Y6 + (m16 + m17);
    O[5] = X4 + Z8 + (m18 - m16);
    O[6] = X4 - Z8 - (m16 + m18);
    O[7] = Y6 + Z8 + (m17 - m18);
    O[8] = Y6 - Z8 + (m17 + m18);
}

// e.(x, y, z) for a compile-time e with components in {-1, 0, 1}, written
// without multiplications by the constants: IEEE arithmetic does not fold
// 0 * x or x + 0, so the plain dot product would spend instructions on them.
template <int CX, int CY, int CZ, class R>
__host__ __device__ __forceinline__ R dot_e(R x, R y, R z) {
    if constexpr (CX != 0) {
        R s = CX > 0 ? x : -x;
        if constexpr (CY != 0) s = CY > 0 ? s + y : s - y;
        if constexpr (CZ != 0) s = CZ > 0 ? s + z : s - z;
        return s;
    } else if constexpr (CY != 0) {
        R s = CY > 0 ? y : -y;
        if constexpr (CZ != 0) s = CZ > 0 ? s + z : s - z;
        return s;
    } else if constexpr (CZ != 0) {
        return CZ > 0 ? z : -z;
    } else {
        return (R)0;
    }
}

// Signed sums over opposite pairs: acc[d] = sum_p e_d(2p+1) v[p] over the
// pairs with e_d != 0 (and, with CLS >= 0, only pairs of weight class CLS:
// 0 = the class of direction 1, 1 = the others).  The first contributing
// term initialises the sum, so no 0 + x is issued.
template <int LAT>
__host__ __device__ constexpr int pair_e(int p, int d) {
    using L = Lat<LAT>;
    return d == 0 ? L::ex[2 * p + 1] : (d == 1 ? L::ey[2 * p + 1] : L::ez[2 * p + 1]);
}
template <int LAT>
__host__ __device__ constexpr bool pair_in(int p, int cls) {
    return cls < 0 || ((Lat<LAT>::w(2 * p + 1) == Lat<LAT>::w(1)) == (cls == 0));
}
template <int LAT>
__host__ __device__ constexpr int first_pair(int d, int cls) {
    for (int p = 0; p < (Lat<LAT>::Q - 1) / 2; ++p)
        if (pair_in<LAT>(p, cls) && pair_e<LAT>(p, d) != 0) return p;
    return -1;
}
template <int LAT, int CLS, class R, int NP>
__device__ __forceinline__ void pair_sums(const R (&v)[NP], R (&acc)[3]) {
#pragma unroll
    for (int d = 0; d < 3; ++d) acc[d] = (R)0;
    sfor<3>([&](auto D) {
        constexpr int d = decltype(D)::value;
        sfor<NP>([&](auto PI) {
            constexpr int p = decltype(PI)::value;
            constexpr int e = pair_e<LAT>(p, d);
            if constexpr (e != 0 && pair_in<LAT>(p, CLS)) {
                if constexpr (p == first_pair<LAT>(d, CLS)) acc[d] = e > 0 ? v[p] : -v[p];
                else acc[d] = e > 0 ? acc[d] + v[p] : acc[d] - v[p];
            }
        });
    });
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
// FP32 populations, FP64 arithmetic (values widen on load, round on store)
template <> struct Store<ST_F32D> {
    using S = float;
    using R = double;
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
    int wet_uniform;       // 1: the wetting parameter is wet_val[k] at every node
    R wet_val[2];
    int common_u;          // two components: common equilibrium velocity
    int has_zc;            // any A_kk != 0
    R omega[2];            // 1/tau
    R srate[2][19];        // MRT: s_m / |row m|^2
    R eos_a[2], eos_b[2], eos_RT[2], alpha[2], ginv[2];  // ginv = 1/g_kk
    R A[2];
    R g[2][2];
    R body[3];
    R rho_min[2], rho_max[2];
    R kq[2];               // surface-tension source (D2Q9 MRT): kappa_k g_kk
    R res_rho[2][2];       // open boundaries: density of component k in reservoir r
    R res_abb[2][2];       // ... in the inflow of the streaming the pull completes
};

// Neighbour-word bits above the direction bits (bit 0: the node is not
// fluid; bit i: the source x - e_i is solid or a reservoir, so the pull takes
// the node's own opposite population).  Reservoir nodes fill whole planes of
// the marching axis c, so a fluid node next to one takes from it exactly the
// directions with e_c = +1 (reservoir plane below) or e_c = -1 (above).
constexpr uint32_t NW_RES_LO = 1u << 20;   // plane c - 1 is a reservoir
constexpr uint32_t NW_RES_HI = 1u << 21;   // plane c + 1 is a reservoir
constexpr uint32_t NW_RES_ID = 1u << 22;   // ... and it is reservoir 1
constexpr uint32_t NW_OWN_RES = 1u << 23;  // the node is a reservoir node
constexpr uint32_t NW_OWN_ID = 1u << 24;   // ... of reservoir 1
constexpr uint32_t NW_OWN_CONV = 1u << 25; // the node is in the convective outlet plane

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
//
// The plane index c is the same for every lane of a wavefront (a workgroup
// works on one plane at a time), so the address of a population splits into
// a wavefront-uniform 64-bit base (array, component, direction, source plane:
// scalar registers and scalar ALU) and a 32-bit per-lane offset inside the
// plane.  The in-plane offset of the source x - e_i depends only on
// (e_a, e_b), so nine adds cover all directions and each load costs one
// vector instruction besides itself.
// ---------------------------------------------------------------------------
// BBI: take the bounce-back source at issue time (two components, where every
// gather pays a full memory latency) or patch it after the streaming loads
// (one component: a cheaper plain path for the bulk).
// RING (deviation storage): the source densities rho* come from an LDS ring
// of the caller, so the pull loads only the 16-bit deviations and finish()
// leaves 1 + h_i for the caller to scale by w_i rho*(source).
template <int LAT, int ST, int NC, bool BBI = (NC > 1), bool RING = false>
struct Pull {
    using L = Lat<LAT>;
    using SS = Store<ST>;
    using S = typename SS::S;
    using R = typename SS::R;
    static constexpr int Q = L::Q;
    S v[NC][Q];
    float rs[NC][SS::DEV && !RING ? Q : 1];

    // Issue the loads of node (a, b, c): f_i(x) = f*_i(x - e_i), or, where
    // x - e_i is solid (bit i of the neighbour word), the halfway bounce-back
    // f*_opp(i)(x).  With BBI the source is chosen per lane before the load,
    // so a node next to a wall costs no second, dependent round of loads (a
    // wavefront with no such lane takes the plain path); without it the
    // streaming loads are issued unconditionally and finish() replaces the
    // values that came from solid nodes.
    __device__ __forceinline__ void issue(const StepArgs<R>& P, int a, int b, int c, uint32_t word) {
        const int NA = P.NA, NB = P.NB, NCc = P.NC_;
        const size_t plane = (size_t)NA * NB;
        // the direction stride is made opaque here so that the per-direction
        // bases are formed in the loop by the scalar unit instead of being
        // kept live across it (which spills scalar registers)
        size_t N = (size_t)P.N;
        asm volatile("" : "+s"(N));
        // source coordinate x - e for e = -1, 0, +1 (index e + 1), periodic
        const uint32_t col[3] = {(uint32_t)(a == NA - 1 ? 0 : a + 1), (uint32_t)a,
                                 (uint32_t)(a == 0 ? NA - 1 : a - 1)};
        const uint32_t row[3] = {(uint32_t)((b == NB - 1 ? 0 : b + 1) * NA), (uint32_t)(b * NA),
                                 (uint32_t)((b == 0 ? NB - 1 : b - 1) * NA)};
        const size_t cs[3] = {(size_t)(c == NCc - 1 ? 0 : c + 1), (size_t)c, (size_t)(c == 0 ? NCc - 1 : c - 1)};
        const char* fb = reinterpret_cast<const char*>(P.fin);
        [[maybe_unused]] const char* rb = reinterpret_cast<const char*>(P.rin);
        auto load = [&](int k, int dir, size_t pl, uint32_t e, int i) {
            v[k][i] = *reinterpret_cast<const S*>(fb + ((size_t)(k * Q + dir) * N + pl) * sizeof(S) +
                                                  e * (uint32_t)sizeof(S));
            if constexpr (SS::DEV && !RING)
                rs[k][i] = *reinterpret_cast<const float*>(rb + ((size_t)k * N + pl) * 4 + e * 4u);
        };
        const bool wall = BBI && __builtin_amdgcn_ballot_w64((word & ~1u) != 0u) != 0;
        sfor<Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            // keep offsets 32-bit values computed here: hoisted out of the plane
            // loop they would be widened to 64 bits and the loads would lose the
            // scalar-base addressing form
            uint32_t e = row[L::eb(i) + 1] + col[L::ea(i) + 1];
            asm volatile("" : "+v"(e));
            const size_t pl = cs[L::ec(i) + 1] * plane;
            if (i == 0 || !wall) {
#pragma unroll
                for (int k = 0; k < NC; ++k) load(k, i, pl, e, i);
            } else if (!((word >> i) & 1u)) {
#pragma unroll
                for (int k = 0; k < NC; ++k) load(k, i, pl, e, i);
            } else {
                uint32_t eo = row[1] + col[1];
                asm volatile("" : "+v"(eo));
#pragma unroll
                for (int k = 0; k < NC; ++k) load(k, opp(i), cs[1] * plane, eo, i);
            }
        });
    }

    // Conversion to the compute type (and, without BBI, the bounce-back
    // loads after the streaming ones).
    __device__ __forceinline__ void finish(const StepArgs<R>& P, int a, int b, int c, uint32_t word,
                                           R (&f)[NC][Q]) {
        if (!BBI && (word & ~1u)) {
            const size_t plane = (size_t)P.NA * P.NB;
            const size_t N = (size_t)P.N;
            uint32_t e = (uint32_t)(b * P.NA + a);
            asm volatile("" : "+v"(e));
            const size_t pl = (size_t)c * plane;
            const char* fb = reinterpret_cast<const char*>(P.fin);
            [[maybe_unused]] const char* rb = reinterpret_cast<const char*>(P.rin);
            sfor<Q - 1>([&](auto I) {
                constexpr int i = decltype(I)::value + 1;
                if ((word >> i) & 1u) {
#pragma unroll
                    for (int k = 0; k < NC; ++k) {
                        v[k][i] = *reinterpret_cast<const S*>(fb + ((size_t)(k * Q + opp(i)) * N + pl) * sizeof(S) +
                                                              e * (uint32_t)sizeof(S));
                        if constexpr (SS::DEV && !RING)
                            rs[k][i] = *reinterpret_cast<const float*>(rb + ((size_t)k * N + pl) * 4 + e * 4u);
                    }
                }
            });
        }
        sfor<Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                if constexpr (SS::DEV && RING) f[k][i] = 1.0f + SS::load(v[k][i]);
                else if constexpr (SS::DEV) f[k][i] = (float)L::w(i) * rs[k][i] * (1.0f + SS::load(v[k][i]));
                else f[k][i] = (R)v[k][i];
            }
        });
    }
};

template <int LAT, int ST, int NC>
__device__ __forceinline__ void pull_node(const StepArgs<typename Store<ST>::R>& P, int a, int b, int c,
                                          uint32_t word, typename Store<ST>::R (&f)[NC][Lat<LAT>::Q]) {
    Pull<LAT, ST, NC> pu;
    pu.issue(P, a, b, c, word);
    pu.finish(P, a, b, c, word, f);
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
        R p;
        if constexpr (std::is_same<R, float>::value) {
            // hardware reciprocal and square root (1 ulp each) in single precision
            const float io = __builtin_amdgcn_rcpf(om);
            p = rho * P.eos_RT[k] * ((R)1 + eta + eta * eta - eta * eta * eta) * (io * io * io) -
                P.eos_a[k] * rho * rho;
        } else {
            p = rho * P.eos_RT[k] * ((R)1 + eta + eta * eta - eta * eta * eta) / (om * om * om) -
                P.eos_a[k] * rho * rho;
        }
        const R u = P.alpha[k] * p - rho * (R)(1.0 / 3.0);
        R arg = (R)2 * u * P.ginv[k];
        arg = arg > (R)0 ? arg : (R)0;
        if constexpr (std::is_same<R, float>::value) psi = __builtin_amdgcn_sqrtf(arg);
        else psi = sqrt(arg);
        U = u;
    } else {
        psi = rho;
        U = (R)0;
    }
}

// ---------------------------------------------------------------------------
// Open boundary (anti-bounce-back): a population whose source is a reservoir
// was pulled as the node's own opposite post-collision one, f*_opp(i)(x); it
// becomes 2 w_i rho_res - f*_opp(i)(x), which holds the density halfway
// between the reservoir and x at rho_res (the constant-pressure inlet and
// outlet of Sec. 3.4.3).
// ---------------------------------------------------------------------------
template <int LAT, int NC, class R>
__device__ __forceinline__ void open_fix(const StepArgs<R>& P, uint32_t word, R (&f)[NC][Lat<LAT>::Q]) {
    using L = Lat<LAT>;
    if (!(word & (NW_RES_LO | NW_RES_HI))) return;
    const int side = (word & NW_RES_LO) ? 1 : -1;
    const int id = (word & NW_RES_ID) ? 1 : 0;
    sfor<L::Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if constexpr (L::ec(i) != 0) {
            if (L::ec(i) == side) {
#pragma unroll
                for (int k = 0; k < NC; ++k) f[k][i] = (R)(2.0 * L::w(i)) * P.res_abb[id][k] - f[k][i];
            }
        }
    });
}

// Density a non-fluid node shows its neighbours in the rho ring: a
// reservoir's fixed density, else the solid marks (-1: its virtual density is
// needed, -2: no fluid neighbour).
// A convective outlet node (the last plane of the marching axis) takes the
// density of the node below it, which the ring holds one slot back (`below`;
// a solid mark there gives reservoir 1's density).
template <class R>
__device__ __forceinline__ R nonfluid_rho(const StepArgs<R>& P, uint32_t word, int k, R mark, R below) {
    if (word & NW_OWN_CONV) return below >= (R)0 ? below : P.res_rho[1][k];
    return (word & NW_OWN_RES) ? P.res_rho[(word & NW_OWN_ID) ? 1 : 0][k] : mark;
}

// ---------------------------------------------------------------------------
// The fused step (MOM = false) or the moment evaluation (MOM = true).
// ---------------------------------------------------------------------------
// Post-collision populations are stored nontemporal: they are read again only
// in the next step, after the whole lattice has passed through L2, so caching
// them would only evict the current plane's halo rows (3-4 % faster steps).
#ifndef LBM_NT_STORE
#define LBM_NT_STORE 1
#endif
// Minimum waves per SIMD the register allocator must allow (1: no bound).
// The one-component FP32 kernels fit three waves by themselves and FP64 would
// spill.  The one-component deviation-storage kernels are held to three (MRT
// otherwise takes 171 registers and runs two waves; bounded, it spills two
// and runs 9 % faster).  Bounds on the two-component kernels (three waves for
// deviation storage, four for FP32) measured 16 % slower and no faster.
// Two-component deviation storage in 3-D takes the source densities rho* of
// its pulls from an LDS ring of rho* planes (tile plus halo 3) instead of one
// global load per pulled value (1-3 % faster).  With one component the ring
// pushes the register-bound kernel into spills and runs 23 % slower, so it
// keeps the global loads.
#ifndef LBM_DEV_RING
#define LBM_DEV_RING 1
#endif
#ifndef LBM_ISSUE_PRIO
#define LBM_ISSUE_PRIO 3  // wave priority while a plane's loads are issued together
#endif
#ifndef LBM_WAVES_1C_DEV
#define LBM_WAVES_1C_DEV 3
#endif
template <int NC, int ST>
constexpr int waves_bound() {
    return (ST == ST_F16 || ST == ST_BF16) && NC == 1 ? LBM_WAVES_1C_DEV : 1;
}

template <int LAT, int NC, int ST, int COLL, bool MOM, int TA, int TB, bool CARRY>
__global__ void __launch_bounds__(TA* TB) __attribute__((amdgpu_waves_per_eu(waves_bound<NC, ST>())))
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

    __shared__ uint32_t s_word[3][NT];  // own-node neighbour words of the carried planes
    __shared__ R s_rho[5][NC][RP];  // rho of fluid nodes, -1 at solid nodes
    __shared__ R s_psi[3][NC][PP];
    __shared__ R s_U[3][NC][PP];
    // rho* ring (deviation storage, 3-D): planes c-1, c, c+1 of the plane being
    // pulled and the one fetched ahead, over the tile with halo 3 (the sources
    // of the halo-2 positions)
    constexpr bool RSR = SS::DEV && D3 && NC == 2 && LBM_DEV_RING;
    constexpr int SWA = TA + 6, SWB = TB + 6, SP = SWA * SWB;
    constexpr int RLD = RSR ? (SP + NT - 1) / NT : 1;
    __shared__ float s_rs[RSR ? 4 : 1][NC][RSR ? SP : 1];

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

    // Solid positions are marked in the rho ring: -1 for a solid node with a
    // fluid neighbour (its virtual density is needed), -2 for one whose
    // neighbours are all solid (its pseudopotential is never read).
    constexpr uint32_t ALLNB = ((1u << Q) - 1u) & ~1u;
    auto solid_mark = [](uint32_t word) { return (word & ALLNB) == ALLNB ? (R)-2 : (R)-1; };

    // ---- phase 1: pull a plane with halo 2, store rho (solid: < 0) --------
    // Each thread pulls its own node (kept in registers until its collision
    // two planes later when CARRY) and HPT halo positions.  A halo-2 position
    // (outside the psi halo) only feeds virtual densities and is pulled only
    // when it has a solid neighbour.  The neighbour words of the next plane
    // are fetched one plane ahead so that no pull waits for them.
    const int la_own = tid % TA, lb_own = tid / TA;
    const int own_idx = (lb_own + H2B) * RWA + la_own + 2;
    constexpr int HALO = RP - NT;
    constexpr int HPT = (HALO + NT - 1) / NT;
    constexpr int H1N = D3 ? 2 * (TA + 2) + 2 * TB : 0;  // psi-ring positions (3-D)
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
        if constexpr (D3) {
            // the psi ring (halo 1) first, on the lowest threads, then halo 2
            if (hh < H1N) {
                if (hh < TA + 2) {
                    rb = 1;
                    ra = 1 + hh;
                } else if (hh < 2 * (TA + 2)) {
                    rb = TB + 2;
                    ra = 1 + hh - (TA + 2);
                } else {
                    const int h3 = hh - 2 * (TA + 2);
                    rb = 2 + h3 / 2;
                    ra = (h3 & 1) ? TA + 2 : 1;
                }
            } else {
                const int g = hh - H1N;
                if (g < RWA) {
                    rb = 0;
                    ra = g;
                } else if (g < 2 * RWA) {
                    rb = RWB - 1;
                    ra = g - RWA;
                } else {
                    const int g3 = g - 2 * RWA;
                    rb = 1 + g3 / 2;
                    ra = (g3 & 1) ? RWA - 1 : 0;
                }
            }
        } else if (hh < TOP) {
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
    // rho* ring (RSR): fetch plane cp of the tile with halo 3 into registers,
    // store it into its slot; scale pulled 1 + h_i by w_i rho*(x - e_i)
    const bool smallSA = NA < SWA, smallSB = NB < SWB;
    auto rs_fetch = [&](int cp, float(&r)[NC][RLD]) {
        const int c = wrap_c(cp);
#pragma unroll
        for (int j = 0; j < RLD; ++j) {
            const int idx = tid + j * NT;
            if (idx < SP) {
                int ga = a0 + idx % SWA - 3, gb = b0 + idx / SWA - 3;
                ga = smallSA ? wrap_any(ga, NA) : wrap_near(ga, NA);
                gb = smallSB ? wrap_any(gb, NB) : wrap_near(gb, NB);
                const size_t n = ((size_t)c * NB + gb) * NA + ga;
#pragma unroll
                for (int k = 0; k < NC; ++k) r[k][j] = P.rin[(size_t)k * N + n];
            }
        }
    };
    auto rs_store = [&](int cp, const float(&r)[NC][RLD]) {
        const int sl = (cp - c0 + 8) & 3;
#pragma unroll
        for (int j = 0; j < RLD; ++j) {
            const int idx = tid + j * NT;
            if (idx < SP) {
#pragma unroll
                for (int k = 0; k < NC; ++k) s_rs[sl][k][idx] = r[k][j];
            }
        }
    };
    auto rs_scale = [&](R(&f)[NC][Q], uint32_t word, int lofs, int cp) {
        // flat offsets into s_rs of the own position in the planes cp - 1, cp, cp + 1
        const int o0 = ((cp - c0 + 8) & 3) * NC * SP + lofs;
        const int on = ((cp + 1 - c0 + 8) & 3) * NC * SP + lofs;
        const int op = ((cp - 1 - c0 + 8) & 3) * NC * SP + lofs;
        const float* ring = &s_rs[0][0][0];
        sfor<Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            // source x - e_i: plane cp + 1 for e_c = -1, cp - 1 for e_c = +1;
            // a bounced population comes from the node itself
            const int src = (L::ec(i) == 0 ? o0 : (L::ec(i) < 0 ? on : op)) - L::eb(i) * SWA - L::ea(i);
            const int at = (i != 0 && ((word >> i) & 1u)) ? o0 : src;
#pragma unroll
            for (int k = 0; k < NC; ++k) f[k][i] = ((float)L::w(i) * ring[at + k * SP]) * f[k][i];
        });
    };

    auto fill_rho = [&](int cp, R(&fo)[NC][Q]) {
        const int slot = (cp - c0 + 5) % 5;
        const int bslot = (cp - c0 + 4) % 5;  // plane cp - 1 (an outlet plane is never the first of the ring)
        const int c = wrap_c(cp);
        const uint32_t wo = w_own;
        s_word[(cp - c0 + 3) % 3][tid] = wo;  // read back by this thread at the plane's collision
        uint32_t wh[HPT];
#pragma unroll
        for (int j = 0; j < HPT; ++j) wh[j] = w_halo[j];
        fetch_words(cp + 1);
        // A halo position is pulled unless it is solid, or it lies on the
        // outer ring (halo 2, which feeds only virtual densities) without a
        // solid neighbour.
        auto need = [&](int j) { return h_on[j] && !(wh[j] & 1u) && !(h_outer[j] && wh[j] == 0u); };
        // With plain storage and one component all loads of the plane are
        // issued before any is waited for, so the halo pulls do not add a
        // second memory latency.  Deviation storage (which also loads rho* per
        // direction) and two components (twice the values per node) keep the
        // sequential order: with several nodes in flight they lose a wave per
        // SIMD, which costs more than the latency saved.
        constexpr bool OVERLAP = !SS::DEV && NC == 1;
        // the rho* plane two ahead is fetched first, so that storing it waits
        // only for its own loads
        float rsn[NC][RLD];
        if constexpr (RSR) rs_fetch(cp + 2, rsn);
        Pull<LAT, ST, NC, (NC > 1), RSR> po;
        Pull<LAT, ST, NC, (NC > 1), RSR> ph[OVERLAP ? HPT : 1];
        // A solid node holds no populations: its lane issues no loads (a
        // wavefront of solid nodes skips the pull), and its registers are
        // never read, since the ring marks it solid and its collision returns.
        // (two components only: with one component the branch would split the
        // overlapped own-node and halo loads, which costs more than the few
        // solid lanes of its workloads save)
        const bool own_fluid = NC == 1 || !(wo & 1u);
        // While it issues the plane's loads together the wave runs at raised
        // priority, so that they leave before other waves' arithmetic (one
        // component: 1.5 % faster; the sequential two-component pulls ran 26 %
        // slower with it).
        if constexpr (OVERLAP) __builtin_amdgcn_s_setprio(LBM_ISSUE_PRIO);
        if (own_fluid) po.issue(P, own_a, own_b, c, wo);
        if constexpr (OVERLAP) {
#pragma unroll
            for (int j = 0; j < HPT; ++j)
                if (need(j)) ph[j].issue(P, h_a[j], h_b[j], c, wh[j]);
            __builtin_amdgcn_s_setprio(0);
        }
        if constexpr (RSR) rs_store(cp + 2, rsn);
        if (own_fluid) po.finish(P, own_a, own_b, c, wo, fo);
        if constexpr (RSR)
            if (!(wo & 1u)) rs_scale(fo, wo, (lb_own + 3) * SWA + la_own + 3, cp);
        if (wo & 1u) {
#pragma unroll
            for (int k = 0; k < NC; ++k)
                s_rho[slot][k][own_idx] = nonfluid_rho(P, wo, k, solid_mark(wo), s_rho[bslot][k][own_idx]);
        } else {
            open_fix<LAT, NC>(P, wo, fo);
#pragma unroll
            for (int k = 0; k < NC; ++k) s_rho[slot][k][own_idx] = rho_sum(fo, k);
        }
#pragma unroll
        for (int j = 0; j < HPT; ++j) {
            if (!h_on[j]) continue;
            if (wh[j] & 1u) {
#pragma unroll
                for (int k = 0; k < NC; ++k)
                    s_rho[slot][k][h_idx[j]] = nonfluid_rho(P, wh[j], k, solid_mark(wh[j]), s_rho[bslot][k][h_idx[j]]);
            } else if (!need(j)) {
#pragma unroll
                for (int k = 0; k < NC; ++k) s_rho[slot][k][h_idx[j]] = (R)0;  // never read
            } else {
                R f[NC][Q];
                if constexpr (OVERLAP) {
                    ph[j].finish(P, h_a[j], h_b[j], c, wh[j], f);
                } else {
                    ph[0].issue(P, h_a[j], h_b[j], c, wh[j]);
                    ph[0].finish(P, h_a[j], h_b[j], c, wh[j], f);
                }
                if constexpr (RSR) {
                    // ring position (ra + 1, rb + 1) of halo position (ra, rb)
                    const int rb = h_idx[j] / RWA;
                    rs_scale(f, wh[j], h_idx[j] + 2 * rb + SWA + 1, cp);
                }
                open_fix<LAT, NC>(P, wh[j], f);
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
            if (r0 == (R)-2) {
                // solid without fluid neighbours
#pragma unroll
                for (int k = 0; k < NC; ++k) {
                    s_psi[pslot][k][idx] = 0;
                    s_U[pslot][k][idx] = 0;
                }
            } else if (r0 >= (R)0) {
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
                        const R prm = P.wet_uniform ? P.wet_val[k] : P.wet[(size_t)k * N + n];
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
    auto collide_f = [&](int c, const R(&f)[NC][Q], bool pulled, uint32_t wpull) {
        const int la = la_own, lb = lb_own;
        const int a = a0 + la, b = b0 + lb;
        if (a >= NA || b >= NB) return;
        const int n = (c * NB + b) * NA + a;
        // with the carry, the neighbour word came with the pull of this plane
        const uint32_t word = pulled ? wpull : s_word[(c - c0 + 3) % 3][tid];
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
        constexpr int NP = (Q - 1) / 2;
        R rho[NC], j[NC][3];
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            R r = f[k][0], dl[NP];
            sfor<NP>([&](auto PI) {
                constexpr int p = decltype(PI)::value;
                constexpr int i = 2 * p + 1;  // e_{i+1} = -e_i
                r += f[k][i] + f[k][i + 1];
                dl[p] = f[k][i] - f[k][i + 1];
            });
            rho[k] = r;
            pair_sums<LAT, -1>(dl, j[k]);
        }
        // interaction force (Eq. 13) with G_i = w_i / c_s^2.  The sums over
        // directions are taken as differences across opposite neighbours,
        // psi(x + e_i) - psi(x - e_i), gathered per weight class and scaled
        // once per class: D^kk = sum_i G_i psi^kk(x + e_i) e_i.
        const int sc = (c - c0 + 3) % 3;
        const int pc = (lb + H1B) * PWA + la + 1;
        constexpr R G0 = (R)(3.0 * L::w(1));                // class of direction 1
        constexpr R G1 = (R)(3.0 * L::w(Q - 1));            // the other class
        auto gather = [&](const R(&ring)[3][NC][PP], int kk, R(&out)[3]) {
            R dv[NP];
            sfor<NP>([&](auto PI) {
                constexpr int i = 2 * decltype(PI)::value + 1;
                const int slp = (c + L::ec(i) - c0 + 3) % 3;
                const int slm = (c - L::ec(i) - c0 + 3) % 3;
                const int offp = pc + L::eb(i) * PWA + L::ea(i);
                const int offm = pc - L::eb(i) * PWA - L::ea(i);
                dv[decltype(PI)::value] = ring[slp][kk][offp] - ring[slm][kk][offm];
            });
            R s0[3], s1[3];
            pair_sums<LAT, 0>(dv, s0);
            pair_sums<LAT, 1>(dv, s1);
            sfor<3>([&](auto D) {
                constexpr int d = decltype(D)::value;
                constexpr bool h0 = first_pair<LAT>(d, 0) >= 0, h1 = first_pair<LAT>(d, 1) >= 0;
                if constexpr (h0 && h1) out[d] = G0 * s0[d] + G1 * s1[d];
                else if constexpr (h0) out[d] = G0 * s0[d];
                else if constexpr (h1) out[d] = G1 * s1[d];
                else out[d] = (R)0;
            });
        };
        R Dps[NC][3];
#pragma unroll
        for (int kk = 0; kk < NC; ++kk) gather(s_psi, kk, Dps[kk]);
        R F[NC][3];
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            const R psik = s_psi[sc][k][pc];
            const R Bk = (R)1 - P.A[k];
            R sv[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                R t = P.g[k][0] * Dps[0][d];
#pragma unroll
                for (int kk = 1; kk < NC; ++kk) t += P.g[k][kk] * Dps[kk][d];
                sv[d] = t;
            }
            const R cpsi = -Bk * psik;
            F[k][0] = cpsi * sv[0] + rho[k] * P.body[0];
            F[k][1] = cpsi * sv[1] + rho[k] * P.body[1];
            F[k][2] = cpsi * sv[2] + rho[k] * P.body[2];
            if (P.has_zc) {
                R zu[3];
                gather(s_U, k, zu);
                F[k][0] -= P.A[k] * zu[0];
                F[k][1] -= P.A[k] * zu[1];
                F[k][2] -= P.A[k] * zu[2];
            }
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
                // Opposite directions i, i+1 (e_{i+1} = -e_i) share the even part
                // of f^eq and of the forcing term and negate the odd part:
                //   f^eq_i     = w rho (1 + 4.5 (e.u)^2 - 1.5 u^2) +- 3 w rho e.u
                //   dF_i (Eq. 5) = f^eq_i(rho, u + du) - f^eq_i(rho, u)
                //              = w rho (4.5 e.du (2 e.u + e.du) - 1.5 (2 u.du + du^2)) +- 3 w rho e.du
                // (expanded so that no two O(w rho) numbers are subtracted).  Every
                // term is formed as w rho times a bracket that holds only the
                // velocity-dependent part, and w rho (one product per weight class)
                // enters once, through a fused multiply-add: in single precision a
                // population then carries two roundings at its own magnitude instead
                // of four to seven, which is what limits the accuracy of long runs
                // whose slow modes integrate the per-step rounding.
                [[maybe_unused]] const R wr0 = (R)L::w(0) * r;  // rest
                const R wrA = (R)L::w(1) * r;                 // class of direction 1
                const R wrB = (R)L::w(Q - 1) * r;             // the other class
                auto wr_of = [&](auto PI) -> R {
                    return pair_in<LAT>(decltype(PI)::value, 0) ? wrA : wrB;
                };
                // even / odd parts of f^eq (q) and of the forcing term (g) of pair p
                auto eq_parts = [&](auto PI, R& qs, R& qa) {
                    constexpr int i = 2 * decltype(PI)::value + 1;
                    const R wr = wr_of(PI);
                    const R eu = dot_e<L::ex[i], L::ey[i], L::ez[i]>(ux, uy, uz);
                    qs = wr + wr * ((R)4.5 * (eu * eu) - usq);
                    qa = wr * ((R)3 * eu);
                };
                auto force_parts = [&](auto PI, R& gs, R& ga) {
                    constexpr int i = 2 * decltype(PI)::value + 1;
                    const R wr = wr_of(PI);
                    const R eu = dot_e<L::ex[i], L::ey[i], L::ez[i]>(ux, uy, uz);
                    const R ed = dot_e<L::ex[i], L::ey[i], L::ez[i]>(dx, dy, dz);
                    gs = wr * ((R)4.5 * ed * ((R)2 * eu + ed) - dsq);
                    ga = wr * ((R)3 * ed);
                };
                R fo[Q];
                if constexpr (COLL == COLL_BGK) {
                    // f* = (1 - omega) f + omega f^eq + dF
                    //    = (1 - omega) f + omega w rho + w rho (s_even +- s_odd)
                    const R om = P.omega[k], om1 = (R)1 - om;
                    const R woA = om * wrA, woB = om * wrB;
                    sfor<NP>([&](auto PI) {
                        constexpr int p = decltype(PI)::value;
                        constexpr int i = 2 * p + 1;
                        const R wr = wr_of(PI);
                        const R wo = pair_in<LAT>(p, 0) ? woA : woB;
                        const R eu = dot_e<L::ex[i], L::ey[i], L::ez[i]>(ux, uy, uz);
                        const R ed = dot_e<L::ex[i], L::ey[i], L::ez[i]>(dx, dy, dz);
                        const R se = om * ((R)4.5 * (eu * eu) - usq) + ((R)4.5 * ed * ((R)2 * eu + ed) - dsq);
                        const R so = (R)3 * (om * eu + ed);
                        fo[i] = om1 * f[k][i] + (wo + wr * (se + so));
                        fo[i + 1] = om1 * f[k][i + 1] + (wo + wr * (se - so));
                    });
                } else if constexpr (COLL == COLL_CLBM) {
                    // Central moments with the consistent forcing (Eq. 3, Eq. 7-8),
                    // one D2Q9 component:
                    //   f* = f + T^-1 [-S T (f - f^eq) + (I - S/2) T R],
                    //   R_i = (F / rho) . (e_i - u) / c_s^2 f^eq_i,  u = (j + F/2) / rho,
                    // T = rows of the moment basis at e_i - u.  With m = M (f - f^eq)
                    // and r = M R the raw moments, T = N M and N = T M^-1 = T M^T
                    // diag(1 / |row|^2) has unit pivots for any |u| < 0.3, so
                    // N v = y is solved without pivoting and f* = f + M^-1 v.
                    static_assert(LAT == LAT_D2Q9, "central moments: D2Q9 only");
                    const R uxc = (j[k][0] + (R)0.5 * F[k][0]) * invr;
                    const R uyc = (j[k][1] + (R)0.5 * F[k][1]) * invr;
                    const R us = (R)1.5 * (uxc * uxc + uyc * uyc);
                    const R uF = uxc * F[k][0] + uyc * F[k][1];
                    R d[Q], Rf[Q];
                    sfor<Q>([&](auto I) {
                        constexpr int i = decltype(I)::value;
                        const R wri = i == 0 ? wr0 : (L::w(i) == L::w(1) ? wrA : wrB);
                        const R eu = dot_e<L::ex[i], L::ey[i], 0>(uxc, uyc, (R)0);
                        const R fe = wri + wri * ((R)3 * eu + (R)4.5 * (eu * eu) - us);
                        d[i] = f[k][i] - fe;
                        Rf[i] = (R)3 * (dot_e<L::ex[i], L::ey[i], 0>(F[k][0], F[k][1], (R)0) - uF) * invr * fe;
                    });
                    // raw moments and the rows of N
                    R m[Q], rr[Q], Nm[Q][Q];
                    sfor<Q>([&](auto A) {
                        constexpr int a = decltype(A)::value;
                        R sm = 0, sr = 0;
                        sfor<Q>([&](auto I) {
                            constexpr int i = decltype(I)::value;
                            constexpr double cf = mrt_coef<LAT>(a, i);
                            if constexpr (cf != 0.0) {
                                sm += (R)cf * d[i];
                                sr += (R)cf * Rf[i];
                            }
                        });
                        m[a] = sm;
                        rr[a] = sr;
                        sfor<Q>([&](auto B) { Nm[a][decltype(B)::value] = (R)0; });
                    });
                    sfor<Q>([&](auto I) {
                        constexpr int i = decltype(I)::value;
                        const R cx = (R)L::ex[i] - uxc, cy = (R)L::ey[i] - uyc;
                        const R c2 = cx * cx + cy * cy;
                        const R row[9] = {(R)1,
                                          (R)-4 + (R)3 * c2,
                                          (R)4 - (R)10.5 * c2 + (R)4.5 * c2 * c2,
                                          cx,
                                          ((R)3 * c2 - (R)5) * cx,
                                          cy,
                                          ((R)3 * c2 - (R)5) * cy,
                                          cx * cx - cy * cy,
                                          cx * cy};
                        sfor<Q>([&](auto B) {
                            constexpr int b = decltype(B)::value;
                            constexpr double cf = mrt_coef<LAT>(b, i) / mrt_norm<LAT>(b);
                            if constexpr (cf != 0.0) {
#pragma unroll
                                for (int a = 0; a < Q; ++a) Nm[a][b] += row[a] * (R)cf;
                            }
                        });
                    });
                    // y = -S N m + (I - S/2) N r, then N v = y by elimination
                    R y[Q];
                    sfor<Q>([&](auto A) {
                        constexpr int a = decltype(A)::value;
                        R z = 0, w2 = 0;
#pragma unroll
                        for (int b = 0; b < Q; ++b) {
                            z += Nm[a][b] * m[b];
                            w2 += Nm[a][b] * rr[b];
                        }
                        const R sa = P.srate[k][a] * (R)mrt_norm<LAT>(a);
                        y[a] = -sa * z + ((R)1 - (R)0.5 * sa) * w2;
                    });
#pragma unroll
                    for (int c = 0; c < Q; ++c) {
                        const R ip = (R)1 / Nm[c][c];
#pragma unroll
                        for (int r = c + 1; r < Q; ++r) {
                            const R l = Nm[r][c] * ip;
#pragma unroll
                            for (int b = c + 1; b < Q; ++b) Nm[r][b] -= l * Nm[c][b];
                            y[r] -= l * y[c];
                        }
                    }
                    R v[Q];
#pragma unroll
                    for (int c = Q - 1; c >= 0; --c) {
                        R t = y[c];
#pragma unroll
                        for (int b = c + 1; b < Q; ++b) t -= Nm[c][b] * v[b];
                        v[c] = t / Nm[c][c];
                    }
                    sfor<Q>([&](auto I) {
                        constexpr int i = decltype(I)::value;
                        R x = 0;
                        sfor<Q>([&](auto B) {
                            constexpr int b = decltype(B)::value;
                            constexpr double cf = mrt_coef<LAT>(b, i) / mrt_norm<LAT>(b);
                            if constexpr (cf != 0.0) x += (R)cf * v[b];
                        });
                        fo[i] = f[k][i] + x;
                    });
                } else {
                    // f* = f - M^-1 S M (f - f^eq) + dF with M^-1 = M^T diag(1/|row|^2)
                    // (folded into srate).  Even rows see only d_i + d_{i+1}, odd
                    // rows only d_i - d_{i+1}.  The density row of f - f^eq is zero,
                    // and so are the momentum rows when f^eq takes u = j / rho (one
                    // component); those rows are skipped.
                    R dp[NP], dm[NP];
                    sfor<NP>([&](auto PI) {
                        constexpr int p = decltype(PI)::value;
                        constexpr int i = 2 * p + 1;
                        R qs, qa;
                        eq_parts(PI, qs, qa);
                        dp[p] = (f[k][i] + f[k][i + 1]) - (R)2 * qs;
                        dm[p] = (f[k][i] - f[k][i + 1]) - (R)2 * qa;
                    });
                    const R d0 = f[k][0] - (wr0 - wr0 * usq);
                    if constexpr (LAT == LAT_D3Q19) {
                        R sr[19], E[NP], O[NP];
#pragma unroll
                        for (int mm = 0; mm < 19; ++mm) sr[mm] = P.srate[k][mm];
                        mrt_pairs_d3q19<R, (NC > 1)>(dp, dm, d0, sr, E, O);
                        sfor<NP>([&](auto PI) {
                            constexpr int p = decltype(PI)::value;
                            constexpr int i = 2 * p + 1;
                            R fs, fa;
                            force_parts(PI, fs, fa);
                            const R as = fs - E[p], aa = fa - O[p];
                            fo[i] = f[k][i] + (as + aa);
                            fo[i + 1] = f[k][i + 1] + (as - aa);
                        });
                    } else {
                    R m[Q];
                    sfor<Q>([&](auto M) {
                        constexpr int mm = decltype(M)::value;
                        constexpr bool skip = mm == 0 || (NC == 1 && mrt_momentum<LAT>(mm));
                        constexpr bool even = mrt_even<LAT>(mm);
                        R s = 0;
                        if constexpr (!skip) {
                            if constexpr (even) {
                                constexpr double c0 = mrt_coef<LAT>(mm, 0);
                                if constexpr (c0 != 0.0) s = (R)c0 * d0;
                            }
                            sfor<NP>([&](auto PI) {
                                constexpr int p = decltype(PI)::value;
                                constexpr double cf = mrt_coef<LAT>(mm, 2 * p + 1);
                                const R x = even ? dp[p] : dm[p];
                                if constexpr (cf == 1.0) s += x;
                                else if constexpr (cf == -1.0) s -= x;
                                else if constexpr (cf != 0.0) s += (R)cf * x;
                            });
                            s *= P.srate[k][mm];
                        }
                        m[mm] = s;
                    });
                    if constexpr (LAT == LAT_D2Q9) {
                        // surface-tension source (Eq. 14-16): C in moment space,
                        // C = [0, 1.5 s_e tr Q, -1.5 s_eps tr Q, 0, 0, 0, 0,
                        //      -s_pxx (Q_xx - Q_yy), -s_pxy Q_xy], with
                        // Q = kappa g [(1 - A) psi sum_i G_i (psi(x + e_i) - psi) e_i e_i
                        //              + (A / 2) sum_i G_i (psi(x + e_i)^2 - psi^2) e_i e_i];
                        // f* = f - M^-1 (S (m - m^eq) - C), and m here already holds
                        // the relaxed moments divided by |row|^2
                        if (P.kq[k] != (R)0) {
                            const R ps = s_psi[sc][k][pc];
                            R sxx = 0, syy = 0, sxy = 0, txx = 0, tyy = 0, txy = 0;
                            sfor<Q - 1>([&](auto I) {
                                constexpr int i = decltype(I)::value + 1;
                                constexpr R Gi = (R)(3.0 * L::w(i));
                                constexpr int ex = L::ex[i], ey = L::ey[i];
                                const R pm = s_psi[(c + L::ec(i) - c0 + 3) % 3][k][pc + L::eb(i) * PWA + L::ea(i)];
                                const R av = Gi * (pm - ps), bv = Gi * (pm * pm - ps * ps);
                                if constexpr (ex != 0) {
                                    sxx += av;
                                    txx += bv;
                                }
                                if constexpr (ey != 0) {
                                    syy += av;
                                    tyy += bv;
                                }
                                if constexpr (ex * ey > 0) {
                                    sxy += av;
                                    txy += bv;
                                } else if constexpr (ex * ey < 0) {
                                    sxy -= av;
                                    txy -= bv;
                                }
                            });
                            const R c1 = P.kq[k] * ((R)1 - P.A[k]) * ps, c2 = P.kq[k] * (R)0.5 * P.A[k];
                            const R Qxx = c1 * sxx + c2 * txx, Qyy = c1 * syy + c2 * tyy;
                            const R Qxy = c1 * sxy + c2 * txy;
                            const R tr = Qxx + Qyy;
                            m[1] -= (R)1.5 * P.srate[k][1] * tr;
                            m[2] += (R)1.5 * P.srate[k][2] * tr;
                            m[7] += P.srate[k][7] * (Qxx - Qyy);
                            m[8] += P.srate[k][8] * Qxy;
                        }
                    }
                    sfor<NP>([&](auto PI) {
                        constexpr int p = decltype(PI)::value;
                        constexpr int i = 2 * p + 1;
                        R se = 0, so = 0;
                        sfor<Q>([&](auto M) {
                            constexpr int mm = decltype(M)::value;
                            constexpr bool skip = mm == 0 || (NC == 1 && mrt_momentum<LAT>(mm));
                            constexpr double cf = mrt_coef<LAT>(mm, i);
                            if constexpr (!skip && cf != 0.0) {
                                R& acc = mrt_even<LAT>(mm) ? se : so;
                                if constexpr (cf == 1.0) acc += m[mm];
                                else if constexpr (cf == -1.0) acc -= m[mm];
                                else acc += (R)cf * m[mm];
                            }
                        });
                        R fs, fa;
                        force_parts(PI, fs, fa);
                        fo[i] = f[k][i] - (se + so) + (fs + fa);
                        fo[i + 1] = f[k][i + 1] - (se - so) + (fs - fa);
                    });
                    }
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
                // store: wavefront-uniform base of (component, direction, plane)
                // plus the 32-bit in-plane offset of the node
                uint32_t e = (uint32_t)(b * NA + a);
                asm volatile("" : "+v"(e));
                const size_t pl = (size_t)c * NA * NB;
                size_t Ns = N;  // opaque: per-direction bases formed here (see pull_node)
                asm volatile("" : "+s"(Ns));
                char* ob = reinterpret_cast<char*>(P.fout);
                // (the base is pinned in scalar registers so that the per-lane part
                // is not folded into a shared 64-bit vector address)
                auto st = [&](char* base, size_t off, auto val) {
                    using T = decltype(val);
                    auto bp = (__attribute__((address_space(1))) char*)(base + off);
                    asm volatile("" : "+s"(bp));
#if LBM_NT_STORE
                    __builtin_nontemporal_store(val, (__attribute__((address_space(1))) T*)(bp + e * (uint32_t)sizeof(T)));
#else
                    *(__attribute__((address_space(1))) T*)(bp + e * (uint32_t)sizeof(T)) = val;
#endif
                };
                if constexpr (SS::DEV) {
                    st(reinterpret_cast<char*>(P.rout), ((size_t)k * Ns + pl) * 4, (float)r);
                    const float ir = 1.0f / r;
                    sfor<Q>([&](auto I) {
                        constexpr int i = decltype(I)::value;
                        constexpr float iw = (float)(1.0 / L::w(i));
                        st(ob, ((size_t)(k * Q + i) * Ns + pl) * sizeof(S), (S)SS::cvt(fo[i] * (iw * ir) - 1.0f));
                    });
                } else {
#pragma unroll
                    for (int i = 0; i < Q; ++i) st(ob, ((size_t)(k * Q + i) * Ns + pl) * sizeof(S), (S)fo[i]);
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
    if constexpr (RSR) {
        // rho* of the planes around the first pulled plane, c0 - 2
        float r[NC][RLD];
        for (int cp = c0 - 3; cp < c0; ++cp) {
            rs_fetch(cp, r);
            rs_store(cp, r);
        }
        __syncthreads();
    }
#pragma nounroll
    for (int it = c0 - 4; it < c1; ++it) {
        fill_rho(it + 2, fc2);
        __syncthreads();
        if (it + 1 >= c0 - 1) fill_psi(it + 1);
        __syncthreads();
        if (it >= c0) {
            if constexpr (CARRY) {
                collide_f(it, fc0, false, 0u);
            } else {
                // re-pull the own node (L2-resident since its ring pull)
                const int a = a0 + la_own, b = b0 + lb_own;
                if (a < NA && b < NB) {
                    const int n = (it * NB + b) * NA + a;
                    const uint32_t word = P.nbr[n];
                    if (!(word & 1u)) {
                        pull_node<LAT, ST, NC>(P, a, b, it, word, fc0);
                        open_fix<LAT, NC>(P, word, fc0);
                    }
                    collide_f(it, fc0, true, word);
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
// Neighbour words from the mask (0 fluid, 1 solid, 2 / 3 reservoir 0 / 1,
// 4 convective outlet): bit 0 = the node is not fluid, bit i = the node
// n - e_i is solid or a reservoir (the pull takes the node's own opposite
// population; an outlet node is pulled from like fluid), and the bits NW_*.
template <int LAT>
__global__ void k_nbr_words(const uint8_t* __restrict__ mask, uint32_t* __restrict__ nbr, int NA,
                            int NB, int NCc) {
    using L = Lat<LAT>;
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    const int N = NA * NB * NCc;
    if (n >= N) return;
    const int a = n % NA, b = (n / NA) % NB, c = n / (NA * NB);
    const uint32_t m0 = mask[n];
    uint32_t w = m0 ? 1u : 0u;
    if (m0 == 2 || m0 == 3) w |= NW_OWN_RES | (m0 == 3 ? NW_OWN_ID : 0u);
    if (m0 == 4) w |= NW_OWN_CONV;
    sfor<L::Q - 1>([&](auto I) {
        constexpr int i = decltype(I)::value + 1;
        const int aa = wrap_any(a - L::ea(i), NA);
        const int bb = wrap_any(b - L::eb(i), NB);
        const int cc = wrap_any(c - L::ec(i), NCc);
        const uint32_t ms = mask[(cc * NB + bb) * NA + aa];
        if (ms && ms != 4) w |= 1u << i;
        if ((ms == 2 || ms == 3) && m0 == 0) w |= (L::ec(i) > 0 ? NW_RES_LO : NW_RES_HI) | (ms == 3 ? NW_RES_ID : 0u);
    });
    nbr[n] = w;
}

// Populations such that the first pull gives f = f^eq(rho0, u0) at every
// fluid node: f*_i(y) = f^eq_i(y + e_i) when y + e_i is fluid, else the
// population bounced back into y, f^eq_opp(i)(y), or, where y + e_i is a
// reservoir, the value 2 w_o rho_res - f^eq_o(y) (o = opp(i)) that the
// anti-bounce-back turns into f^eq_o(y).
struct ResRho {
    double r[2][2];
};
template <int LAT, int NC, int ST>
__global__ void k_init(const typename Store<ST>::R* __restrict__ rho0,
                       const typename Store<ST>::R* __restrict__ u0, const uint32_t* __restrict__ nbr,
                       void* fout, float* rout, int NA, int NB, int NCc, ResRho res) {
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
            if (word & NW_OWN_CONV) {
                // an outlet node holds what streams into y + e_i from it
                const int aa = wrap_any(a + L::ea(i), NA);
                const int bb = wrap_any(b + L::eb(i), NB);
                const int cc = wrap_any(c + L::ec(i), NCc);
                v = feq(k, (cc * NB + bb) * NA + aa, i, L::ex[i], L::ey[i], L::ez[i], L::w(i));
            } else if (!(word & 1u)) {
                // y + e_i lies in a reservoir plane
                const bool to_res = (L::ec(i) < 0 && (word & NW_RES_LO)) || (L::ec(i) > 0 && (word & NW_RES_HI));
                if (to_res) {
                    const R rr = (R)res.r[(word & NW_RES_ID) ? 1 : 0][k];
                    v = (R)(2.0 * L::w(o)) * rr - feq(k, n, o, L::ex[o], L::ey[o], L::ez[o], L::w(o));
                } else if ((word >> o) & 1u && i != 0) {
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

// ---------------------------------------------------------------------------
// Convective outlet (Sec. 3.4.2): after a step that read fin and wrote fout,
// the outlet plane c_o (fluid in the plane c_i = c_o - 1 below it) gets the
// populations that stream into the fluid below at the next pull:
//   g_i = (f_i(x, t) + U f_i(x - c, t + 1)) / (1 + U)     (e_c(i) = -1),
// x = the node below the outlet node, f_i(x, t) = the value this step pulled
// (fin at the outlet node), f_i(x - c, t + 1) = the population streaming into
// the node below x (fout), U = max(0, mean j_c / rho over the fluid of c_i at
// time t).  (The outlet's density, that of the node below it, is filled in
// the rho ring.)  Storage F64 / F32 / F32-with-FP64 arithmetic.
// ---------------------------------------------------------------------------
constexpr int kConvThreads = 256;

// Partial sums (sum u_c, count) of the fluid nodes of plane ci at time t.
template <int LAT, int NC, int ST>
__global__ void __launch_bounds__(kConvThreads)
    k_conv_u(StepArgs<typename Store<ST>::R> P, int ci, double* __restrict__ part) {
    using L = Lat<LAT>;
    using R = typename Store<ST>::R;
    const int plane = P.NA * P.NB;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    double u = 0.0, cnt = 0.0;
    if (t < plane) {
        const int a = t % P.NA, b = t / P.NA;
        const uint32_t word = P.nbr[(size_t)ci * plane + t];
        if (!(word & 1u)) {
            R f[NC][L::Q];
            pull_node<LAT, ST, NC>(P, a, b, ci, word, f);
            open_fix<LAT, NC>(P, word, f);
            double jc = 0.0, r = 0.0;
            for (int k = 0; k < NC; ++k)
                for (int i = 0; i < L::Q; ++i) {
                    r += (double)f[k][i];
                    jc += (double)f[k][i] * L::ec(i);
                }
            u = jc / r;
            cnt = 1.0;
        }
    }
    __shared__ double sh[2][kConvThreads / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        u += __shfl_xor(u, o, 64);
        cnt += __shfl_xor(cnt, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        sh[0][threadIdx.x >> 6] = u;
        sh[1][threadIdx.x >> 6] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double su = 0.0, sc = 0.0;
        for (int w = 0; w < kConvThreads / 64; ++w) {
            su += sh[0][w];
            sc += sh[1][w];
        }
        part[2 * blockIdx.x] = su;
        part[2 * blockIdx.x + 1] = sc;
    }
}

// Ghost populations of the outlet plane co (one thread per outlet node).
template <int LAT, int NC, int ST>
__global__ void __launch_bounds__(kConvThreads)
    k_conv_ghost(StepArgs<typename Store<ST>::R> P, int co, const double* __restrict__ part, int nblk) {
    using L = Lat<LAT>;
    using S = typename Store<ST>::S;
    using R = typename Store<ST>::R;
    constexpr int Q = L::Q;
    const int NA = P.NA, NB = P.NB, NCc = P.NC_;
    const int plane = NA * NB;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= plane) return;
    double su = 0.0, sc = 0.0;  // same order in every thread: one U for the plane
    for (int j = 0; j < nblk; ++j) {
        su += part[2 * j];
        sc += part[2 * j + 1];
    }
    double U = sc > 0.0 ? su / sc : 0.0;
    U = U > 0.0 ? U : 0.0;
    const int a = t % NA, b = t / NA;
    const size_t N = (size_t)P.N;
    const S* fin = reinterpret_cast<const S*>(P.fin);
    S* fout = reinterpret_cast<S*>(P.fout);
    const int ci = wrap_any(co - 1, NCc), cu = wrap_any(co - 2, NCc);
    sfor<Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if constexpr (L::ec(i) == -1) {
            // x = the fluid node this population streams into; xu = the node below x
            const int ax = wrap_any(a + L::ea(i), NA), bx = wrap_any(b + L::eb(i), NB);
            const size_t nx_ = (size_t)ci * plane + bx * NA + ax;
            const size_t nu = (size_t)cu * plane + bx * NA + ax;
            const size_t no = (size_t)co * plane + t;
            if (P.nbr[nx_] & 1u) return;
            const uint32_t wu = P.nbr[nu];
            // f_i(x - c, t + 1): from xu - e_i = the node below this outlet node, or bounced back
            const size_t src = (size_t)ci * plane + t;
            for (int k = 0; k < NC; ++k) {
                const R prev = (R)fin[(size_t)(k * Q + i) * N + no];
                R upw = prev;
                if (!(wu & 1u)) upw = (wu >> i) & 1u ? (R)fout[(size_t)(k * Q + opp(i)) * N + nu]
                                                     : (R)fout[(size_t)(k * Q + i) * N + src];
                fout[(size_t)(k * Q + i) * N + no] = (S)((prev + (R)U * upw) / ((R)1 + (R)U));
            }
        }
    });
}

}  // namespace lbm
