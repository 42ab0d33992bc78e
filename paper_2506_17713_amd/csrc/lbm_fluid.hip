// Fluid-only layout (LBM_LAYOUT_FLUID): the fused Shan-Chen step of the
// dense kernels (streaming with halfway bounce-back, Eq. 1-2; moments, Eq. 4
// and 10; virtual densities at solids, Eq. 17; pseudopotential, Eq. 12;
// interaction force, Eq. 11 and 13; BGK or MRT collision with the
// exact-difference forcing, Eq. 3 and 5; reservoir inflow by
// anti-bounce-back, Sec. 3.4.3) over a list of the fluid nodes.
//
// In a sphere pack at porosity 0.35-0.4 a dense row of 64 nodes holds about
// 25 fluid nodes, and the dense kernel reads whole cache lines of them: about
// 2.5 times the fluid bytes, and three pulls per node (own ring pull, halo
// pulls of the neighbouring tiles, re-pull at the collision).  Here only the
// fluid nodes hold populations, in lattice order, and a step is three
// kernels, two of them passes over the fluid nodes:
//   k_fl_rho    pull, density and psi of every fluid node;
//   k_fl_solid  psi of every solid node next to fluid (virtual density) and
//               of every reservoir node (its fixed density);
//   k_fl_step   pull again, gather psi of the 18 neighbours, force,
//               collision, store.
// Both pulls read the neighbour table (ids of x - e_i), one 4-byte index per
// direction and node; the gather reads psi through the same ids.
//
// Ids: [0, n_col) the fluid nodes, [n_col, n_fl) the nodes of a convective
// outlet plane (pulled from like fluid, never collided), [n_fl, n_sol) the
// solid nodes next to fluid, [n_sol, n_r1) the nodes of reservoir 0 and
// [n_r1, n_ext) those of reservoir 1 (open boundaries, whole planes), each
// range in lattice order.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "lbm_internal.hpp"

using namespace lbm;
using namespace lbmi;

namespace {

constexpr int kFlThreads = 256;
using L = Lat<LAT_D3Q19>;
constexpr int Q = L::Q;
constexpr int NP = (Q - 1) / 2;

// Addresses of the fluid-layout arrays (besides StepArgs).
template <class R>
struct FlArgs {
    const int32_t* tab;   // [Q-1][T]: id of x - e_i (ids >= n_fl: solid or reservoir; -1: not listed)
    const int32_t* dmap;  // [T]: lattice index of id
    const int32_t* emap;  // [N]: id of lattice node, -1 for a solid without fluid neighbour
    // per-id values with the components adjacent ([T][NC]), so that one
    // gather of a neighbour loads every component
    R* rho;               // [T][NC]: density of the fluid ids
    R* psi;               // [T][NC]: psi of every id
    R* U;                 // [T][NC]: U of every id (Zhang-Chen term only)
    int n_col, n_fl, n_sol, n_r1, n_ext, T;
};

// Workgroup b takes ids [256 b, 256 b + 256).  The hardware deals workgroups
// round-robin over the 8 XCDs, so all of them work on neighbouring ids at
// once; mapping consecutive blocks to one XCD instead (contiguous id ranges
// per XCD) measured 4 % slower on the 400^3 pack.

// The NC values of one id, loaded together (one 8- or 16-byte load for two
// components).
template <class R, int NC>
struct Comp {
    R v[NC];
    __device__ __forceinline__ static Comp load(const R* p) {
        Comp c;
        if constexpr (NC == 2) {
            using V = R __attribute__((ext_vector_type(2)));
            const V x = *reinterpret_cast<const V*>(p);
            c.v[0] = x[0];
            c.v[1] = x[1];
        } else {
#pragma unroll
            for (int k = 0; k < NC; ++k) c.v[k] = p[k];
        }
        return c;
    }
};

// Neighbour ids src[i] of x - e_i (src[0] = the node itself) and the pull
// f_i(x) = f*_i(x - e_i), or f*_opp(i)(x) where x - e_i is solid.  With
// deviation storage the stored value is h = f* / (w_i rho*) - 1 with rho*
// the density of the node that stored it ([T][NC] in P.rin), and the pull
// rebuilds f = w_i rho* (1 + h) as the dense kernels do.
template <int NC, int ST>
__device__ __forceinline__ void fl_pull(const StepArgs<typename Store<ST>::R>& P,
                                        const FlArgs<typename Store<ST>::R>& A, int e, int32_t (&src)[Q],
                                        typename Store<ST>::R (&f)[NC][Q]) {
    using SS = Store<ST>;
    using S = typename SS::S;
    using R = typename SS::R;
    const size_t T = (size_t)A.T;
    const S* fin = reinterpret_cast<const S*>(P.fin);
    src[0] = e;
    sfor<Q - 1>([&](auto I) {
        constexpr int i = decltype(I)::value + 1;
        src[i] = A.tab[(size_t)(i - 1) * T + e];
    });
    sfor<Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        // a solid or reservoir source (id >= n_fl, or -1) bounces back the node's own opposite population
        const bool bb = i != 0 && (uint32_t)src[i] >= (uint32_t)A.n_fl;
        const size_t off = bb ? (size_t)opp(i) * T + e : (size_t)i * T + (uint32_t)src[i];
        if constexpr (SS::DEV) {
            const Comp<float, NC> rs = Comp<float, NC>::load(P.rin + (size_t)(bb ? e : src[i]) * NC);
#pragma unroll
            for (int k = 0; k < NC; ++k)
                f[k][i] = (float)L::w(i) * rs.v[k] * (1.0f + SS::load(fin[(size_t)k * Q * T + off]));
        } else {
#pragma unroll
            for (int k = 0; k < NC; ++k) f[k][i] = (R)fin[(size_t)k * Q * T + off];
        }
    });
    if (A.n_sol < A.n_ext) {
        // a reservoir source: anti-bounce-back, 2 w_i rho_res - f*_opp(i)(x),
        // at the density of the streaming this pull completes (Sec. 3.4.3)
        sfor<Q - 1>([&](auto I) {
            constexpr int i = decltype(I)::value + 1;
            if (src[i] >= A.n_sol) {
                const int r = src[i] >= A.n_r1 ? 1 : 0;
#pragma unroll
                for (int k = 0; k < NC; ++k) f[k][i] = (R)(2.0 * L::w(i)) * P.res_abb[r][k] - f[k][i];
            }
        });
    }
}

// rho^k = sum_i f_i, summed as in the dense kernels (rest, then pairs)
template <int NC, class R>
__device__ __forceinline__ R fl_rho_sum(const R (&f)[NC][Q], int k) {
    R r = f[k][0];
    sfor<NP>([&](auto PI) {
        constexpr int i = 2 * decltype(PI)::value + 1;
        r += f[k][i] + f[k][i + 1];
    });
    return r;
}

// Density and momentum (Eq. 4) and the total force (Eq. 11, 13 plus the
// body force) of fluid id e from its pulled populations and the psi (and U)
// of its neighbours, in the operation order of the dense kernels.
template <int NC, class R>
__device__ __forceinline__ void fl_moments_force(const StepArgs<R>& P, const FlArgs<R>& A, int e,
                                                 const int32_t (&src)[Q], const R (&f)[NC][Q], R (&rho)[NC],
                                                 R (&j)[NC][3], R (&F)[NC][3]) {
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        R r = f[k][0], dl[NP];
        sfor<NP>([&](auto PI) {
            constexpr int p = decltype(PI)::value;
            constexpr int i = 2 * p + 1;
            r += f[k][i] + f[k][i + 1];
            dl[p] = f[k][i] - f[k][i + 1];
        });
        rho[k] = r;
        pair_sums<LAT_D3Q19, -1>(dl, j[k]);
    }
    // D^kk = sum_i G_i psi^kk(x + e_i) e_i as differences across opposite
    // neighbours; x + e_i = x - e_opp(i) is src[i + 1] for odd i.  All
    // components of a neighbour come with one load.
    constexpr R G0 = (R)(3.0 * L::w(1));
    constexpr R G1 = (R)(3.0 * L::w(Q - 1));
    auto gather = [&](const R* arr, R(&out)[NC][3]) {
        R dv[NC][NP];
        sfor<NP>([&](auto PI) {
            constexpr int i = 2 * decltype(PI)::value + 1;
            const Comp<R, NC> vp = Comp<R, NC>::load(arr + (size_t)(uint32_t)src[i + 1] * NC);
            const Comp<R, NC> vm = Comp<R, NC>::load(arr + (size_t)(uint32_t)src[i] * NC);
#pragma unroll
            for (int kk = 0; kk < NC; ++kk) dv[kk][decltype(PI)::value] = vp.v[kk] - vm.v[kk];
        });
#pragma unroll
        for (int kk = 0; kk < NC; ++kk) {
            R s0[3], s1[3];
            pair_sums<LAT_D3Q19, 0>(dv[kk], s0);
            pair_sums<LAT_D3Q19, 1>(dv[kk], s1);
#pragma unroll
            for (int d = 0; d < 3; ++d) out[kk][d] = G0 * s0[d] + G1 * s1[d];
        }
    };
    R Dps[NC][3];
    gather(A.psi, Dps);
    R zu[NC][3];
    if (P.has_zc) gather(A.U, zu);
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        const R psik = A.psi[(size_t)e * NC + k];
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
            F[k][0] -= P.A[k] * zu[k][0];
            F[k][1] -= P.A[k] * zu[k][1];
            F[k][2] -= P.A[k] * zu[k][2];
        }
    }
}

// ---------------------------------------------------------------------------
// Pass 1: density and psi of the fluid ids.
// ---------------------------------------------------------------------------
template <int NC, int ST>
__global__ void __launch_bounds__(kFlThreads)
    k_fl_rho(StepArgs<typename Store<ST>::R> P, FlArgs<typename Store<ST>::R> A) {
    using R = typename Store<ST>::R;
    const int e = blockIdx.x * kFlThreads + threadIdx.x;
    if (e >= A.n_col) return;
    int32_t src[Q];
    R f[NC][Q];
    fl_pull<NC, ST>(P, A, e, src, f);
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        const R r = fl_rho_sum<NC>(f, k);
        R ps, u;
        psi_of(P, k, r, ps, u);
        A.rho[(size_t)e * NC + k] = r;
        A.psi[(size_t)e * NC + k] = ps;
        if (P.has_zc) A.U[(size_t)e * NC + k] = u;
    }
}

// ---------------------------------------------------------------------------
// Pass 2: psi of the solid and reservoir ids.  A solid takes the virtual
// density of Eq. 17: the weight-averaged density of its fluid and reservoir
// neighbours x + e_i (in direction order), then phi rho_ave or rho_ave -
// drho, limited to [rho_min, rho_max].  A reservoir node takes its fixed
// density.
// ---------------------------------------------------------------------------
template <int NC, class R>
__global__ void __launch_bounds__(kFlThreads) k_fl_solid(StepArgs<R> P, FlArgs<R> A) {
    const int s = A.n_fl + blockIdx.x * kFlThreads + threadIdx.x;
    if (s >= A.n_ext) return;
    const size_t T = (size_t)A.T;
    if (s >= A.n_sol) {
        const int r = s >= A.n_r1 ? 1 : 0;
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            R ps, u;
            psi_of(P, k, P.res_rho[r][k], ps, u);
            A.psi[(size_t)s * NC + k] = ps;
            if (P.has_zc) A.U[(size_t)s * NC + k] = u;
        }
        return;
    }
    R num[NC], den = 0;
#pragma unroll
    for (int k = 0; k < NC; ++k) num[k] = 0;
    sfor<Q - 1>([&](auto I) {
        constexpr int i = decltype(I)::value + 1;
        const int32_t nb = A.tab[(size_t)(opp(i) - 1) * T + s];  // x + e_i
        if ((uint32_t)nb < (uint32_t)A.n_fl) {
            den += (R)L::w(i);
#pragma unroll
            for (int k = 0; k < NC; ++k) num[k] += (R)L::w(i) * A.rho[(size_t)nb * NC + k];
        } else if (nb >= A.n_sol) {
            const int r = nb >= A.n_r1 ? 1 : 0;
            den += (R)L::w(i);
#pragma unroll
            for (int k = 0; k < NC; ++k) num[k] += (R)L::w(i) * P.res_rho[r][k];
        }
    });
    const int n = A.dmap[s];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        R ps = 0, u = 0;
        if (den > (R)0) {
            const R rave = num[k] / den;
            const R prm = P.wet_uniform ? P.wet_val[k] : P.wet[(size_t)k * P.N + n];
            R rsv = P.wet_drho[k] ? rave - prm : prm * rave;
            rsv = rsv < P.rho_min[k] ? P.rho_min[k] : rsv;
            rsv = rsv > P.rho_max[k] ? P.rho_max[k] : rsv;
            psi_of(P, k, rsv, ps, u);
        }
        A.psi[(size_t)s * NC + k] = ps;
        if (P.has_zc) A.U[(size_t)s * NC + k] = u;
    }
}

// ---------------------------------------------------------------------------
// Pass 3: the fused collision of the fluid ids.  The node collision restates
// that of the dense kernel for D3Q19 (BGK and the MRT pair form), in the same
// operations and order; the dense kernel keeps its own inline copy, whose
// register allocation its tile pipeline is tuned to.
// ---------------------------------------------------------------------------
template <int NC, int ST, int COLL>
__global__ void __launch_bounds__(kFlThreads)
    k_fl_step(StepArgs<typename Store<ST>::R> P, FlArgs<typename Store<ST>::R> A) {
    using S = typename Store<ST>::S;
    using R = typename Store<ST>::R;
    const int e = blockIdx.x * kFlThreads + threadIdx.x;
    if (e >= A.n_col) return;
    const size_t T = (size_t)A.T;
    int32_t src[Q];
    R f[NC][Q];
    fl_pull<NC, ST>(P, A, e, src, f);
    R rho[NC], j[NC][3], F[NC][3];
    fl_moments_force<NC>(P, A, e, src, f, rho, j, F);

    // equilibrium velocity: j / rho, or the common u' of two components
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
    S* out = reinterpret_cast<S*>(P.fout);
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        const R r = rho[k];
        const R invr = (R)1 / r;
        const R ux = ueq[k][0], uy = ueq[k][1], uz = ueq[k][2];
        // du = F / rho; f^eq and the forcing term dF = f^eq(u + du) - f^eq(u)
        // split into the even part shared by opposite directions and the
        // odd part, each as w rho times a velocity bracket
        const R dx = F[k][0] * invr, dy = F[k][1] * invr, dz = F[k][2] * invr;
        const R usq = (R)1.5 * (ux * ux + uy * uy + uz * uz);
        const R dsq = (R)1.5 * ((R)2 * (ux * dx + uy * dy + uz * dz) + dx * dx + dy * dy + dz * dz);
        const R wr0 = (R)L::w(0) * r;
        const R wrA = (R)L::w(1) * r;
        const R wrB = (R)L::w(Q - 1) * r;
        R fo[Q];
        if constexpr (COLL == COLL_BGK) {
            const R om = P.omega[k], om1 = (R)1 - om;
            const R woA = om * wrA, woB = om * wrB;
            sfor<NP>([&](auto PI) {
                constexpr int p = decltype(PI)::value;
                constexpr int i = 2 * p + 1;
                const R wr = pair_in<LAT_D3Q19>(p, 0) ? wrA : wrB;
                const R wo = pair_in<LAT_D3Q19>(p, 0) ? woA : woB;
                const R eu = dot_e<L::ex[i], L::ey[i], L::ez[i]>(ux, uy, uz);
                const R ed = dot_e<L::ex[i], L::ey[i], L::ez[i]>(dx, dy, dz);
                const R se = om * ((R)4.5 * (eu * eu) - usq) + ((R)4.5 * ed * ((R)2 * eu + ed) - dsq);
                const R so = (R)3 * (om * eu + ed);
                fo[i] = om1 * f[k][i] + (wo + wr * (se + so));
                fo[i + 1] = om1 * f[k][i + 1] + (wo + wr * (se - so));
            });
        } else {
            static_assert(COLL == COLL_MRT, "fluid layout: BGK or MRT");
            // f* = f - M^-1 S M (f - f^eq) + dF in the pair form
            R dp[NP], dm[NP];
            sfor<NP>([&](auto PI) {
                constexpr int p = decltype(PI)::value;
                constexpr int i = 2 * p + 1;
                const R wr = pair_in<LAT_D3Q19>(p, 0) ? wrA : wrB;
                const R eu = dot_e<L::ex[i], L::ey[i], L::ez[i]>(ux, uy, uz);
                const R qs = wr + wr * ((R)4.5 * (eu * eu) - usq);
                const R qa = wr * ((R)3 * eu);
                dp[p] = (f[k][i] + f[k][i + 1]) - (R)2 * qs;
                dm[p] = (f[k][i] - f[k][i + 1]) - (R)2 * qa;
            });
            const R d0 = f[k][0] - (wr0 - wr0 * usq);
            R sr[19], E[NP], O[NP];
#pragma unroll
            for (int mm = 0; mm < 19; ++mm) sr[mm] = P.srate[k][mm];
            mrt_pairs_d3q19<R, (NC > 1)>(dp, dm, d0, sr, E, O);
            sfor<NP>([&](auto PI) {
                constexpr int p = decltype(PI)::value;
                constexpr int i = 2 * p + 1;
                const R wr = pair_in<LAT_D3Q19>(p, 0) ? wrA : wrB;
                const R eu = dot_e<L::ex[i], L::ey[i], L::ez[i]>(ux, uy, uz);
                const R ed = dot_e<L::ex[i], L::ey[i], L::ez[i]>(dx, dy, dz);
                const R fs = wr * ((R)4.5 * ed * ((R)2 * eu + ed) - dsq);
                const R fa = wr * ((R)3 * ed);
                const R as = fs - E[p], aa = fa - O[p];
                fo[i] = f[k][i] + (as + aa);
                fo[i + 1] = f[k][i + 1] + (as - aa);
            });
        }
        // the rest population takes the remainder, so that sum_i f*_i = rho
        R m = 0;
        sfor<NP>([&](auto PI) {
            constexpr int i = 2 * decltype(PI)::value + 1;
            m += fo[i] + fo[i + 1];
        });
        fo[0] = r - m;
        if constexpr (Store<ST>::DEV) {
            using SS = Store<ST>;
            const float ir = 1.0f / r;
            sfor<Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                constexpr float iw = (float)(1.0 / L::w(i));
                __builtin_nontemporal_store((S)SS::cvt(fo[i] * (iw * ir) - 1.0f), out + ((size_t)(k * Q + i)) * T + e);
            });
        } else {
#pragma unroll
            for (int i = 0; i < Q; ++i) __builtin_nontemporal_store((S)fo[i], out + ((size_t)(k * Q + i)) * T + e);
        }
    }
    if constexpr (Store<ST>::DEV) {
        // rho* of this node's stored deviations, the components adjacent
#pragma unroll
        for (int k = 0; k < NC; ++k) P.rout[(size_t)e * NC + k] = rho[k];
    }
}

// ---------------------------------------------------------------------------
// Moments in lattice order (Eq. 6, u = (j + F/2) / rho, per component or for
// the mixture), zero at solid nodes: one thread per lattice node.
// ---------------------------------------------------------------------------
template <int NC, int ST>
__global__ void __launch_bounds__(kFlThreads)
    k_fl_mom(StepArgs<typename Store<ST>::R> P, FlArgs<typename Store<ST>::R> A) {
    using R = typename Store<ST>::R;
    const int n = blockIdx.x * kFlThreads + threadIdx.x;
    const size_t N = (size_t)P.N;
    if (n >= P.N) return;
    const int e = A.emap[n];
    if ((uint32_t)e >= (uint32_t)A.n_col) {
        if (P.mom_rho) P.mom_rho[n] = 0;
        if (P.mom_u) {
            P.mom_u[n] = 0;
            P.mom_u[N + n] = 0;
            P.mom_u[2 * N + n] = 0;
        }
        return;
    }
    int32_t src[Q];
    R f[NC][Q];
    fl_pull<NC, ST>(P, A, e, src, f);
    R rho[NC], j[NC][3], F[NC][3];
    fl_moments_force<NC>(P, A, e, src, f, rho, j, F);
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
}

// ---------------------------------------------------------------------------
// Populations whose first pull gives f^eq(rho0, u0) at every fluid node
// (the dense initialisation restricted to fluid ids): f*_i(y) = f^eq_i(y +
// e_i) where y + e_i is fluid, else the population bounced back into y,
// f^eq_opp(i)(y).
// ---------------------------------------------------------------------------
template <int NC, int ST>
__global__ void __launch_bounds__(kFlThreads)
    k_fl_init(const typename Store<ST>::R* __restrict__ rho0, const typename Store<ST>::R* __restrict__ u0,
              FlArgs<typename Store<ST>::R> A, void* fout, float* rout, int N, ResRho res, int NA, int NB, int NCc) {
    using SS = Store<ST>;
    using S = typename SS::S;
    using R = typename SS::R;
    const int e = blockIdx.x * kFlThreads + threadIdx.x;
    if (e >= A.n_fl) return;
    const size_t T = (size_t)A.T;
    S* out = reinterpret_cast<S*>(fout);
    const int n = A.dmap[e];
    auto feq = [&](int k, int m, int ex, int ey, int ez, double wi) -> R {
        const R r = rho0[(size_t)k * N + m];
        const R ux = u0 ? u0[m] : (R)0, uy = u0 ? u0[(size_t)N + m] : (R)0, uz = u0 ? u0[2 * (size_t)N + m] : (R)0;
        const R eu = ex * ux + ey * uy + ez * uz;
        return (R)wi * r * ((R)1 + (R)3 * eu + (R)4.5 * eu * eu - (R)1.5 * (ux * ux + uy * uy + uz * uz));
    };
    if (e >= A.n_col) {
        // an outlet node holds what streams into y + e_i from it (the dense
        // layout's initialisation of outlet nodes; full-precision storage only)
        const int a = n % NA, b = (n / NA) % NB, c = n / (NA * NB);
        for (int k = 0; k < NC; ++k) {
            sfor<Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                const int m = (wrap_any(c + L::ec(i), NCc) * NB + wrap_any(b + L::eb(i), NB)) * NA +
                              wrap_any(a + L::ea(i), NA);
                const R v = feq(k, m, L::ex[i], L::ey[i], L::ez[i], L::w(i));
                if constexpr (!SS::DEV) out[(size_t)(k * Q + i) * T + e] = (S)v;
            });
        }
        return;
    }
    for (int k = 0; k < NC; ++k) {
        const R r0 = rho0[(size_t)k * N + n];
        if constexpr (SS::DEV) rout[(size_t)e * NC + k] = (float)r0;
        sfor<Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            constexpr int o = opp(i);
            R v;
            if (i == 0) {
                v = feq(k, n, 0, 0, 0, L::w(0));
            } else {
                const int32_t nb = A.tab[(size_t)(o - 1) * T + e];  // y + e_i
                if ((uint32_t)nb < (uint32_t)A.n_fl) {
                    v = feq(k, A.dmap[nb], L::ex[i], L::ey[i], L::ez[i], L::w(i));
                } else if (nb >= A.n_sol) {
                    // y + e_i is a reservoir: the value the anti-bounce-back turns into f^eq_o(y)
                    const R rr = (R)res.r[nb >= A.n_r1 ? 1 : 0][k];
                    v = (R)(2.0 * L::w(o)) * rr - feq(k, n, L::ex[o], L::ey[o], L::ez[o], L::w(o));
                } else {
                    v = feq(k, n, L::ex[o], L::ey[o], L::ez[o], L::w(o));
                }
            }
            if constexpr (SS::DEV)
                out[(size_t)(k * Q + i) * T + e] = SS::cvt((float)v / ((float)L::w(i) * (float)r0) - 1.0f);
            else
                out[(size_t)(k * Q + i) * T + e] = (S)v;
        });
    }
}

// Neighbour table: tab[i-1][id] = emap[x_id - e_i] (periodic wrap).
__global__ void __launch_bounds__(kFlThreads)
    k_fl_table(const int32_t* __restrict__ emap, const int32_t* __restrict__ dmap, int32_t* __restrict__ tab,
               int n_ext, int T, int NA, int NB, int NCc) {
    const int e = blockIdx.x * kFlThreads + threadIdx.x;
    if (e >= n_ext) return;
    const int n = dmap[e];
    const int a = n % NA, b = (n / NA) % NB, c = n / (NA * NB);
    sfor<Q - 1>([&](auto I) {
        constexpr int i = decltype(I)::value + 1;
        const int aa = wrap_any(a - L::ea(i), NA);
        const int bb = wrap_any(b - L::eb(i), NB);
        const int cc = wrap_any(c - L::ec(i), NCc);
        tab[(size_t)(i - 1) * T + e] = emap[((size_t)cc * NB + bb) * NA + aa];
    });
}

// ---------------------------------------------------------------------------
// Convective outlet (Sec. 3.4.2), the dense layout's outlet on fluid ids.
// ---------------------------------------------------------------------------
// Density and psi of the outlet ids: those of the node below (reservoir 1's
// density where it is solid), as the dense kernels fill their rho ring.  Runs
// after the fluid densities and before the virtual densities of the solids,
// which average over outlet neighbours too.
template <int NC, class R>
__global__ void __launch_bounds__(kFlThreads) k_fl_conv_rho(StepArgs<R> P, FlArgs<R> A) {
    const int o = A.n_col + blockIdx.x * kFlThreads + threadIdx.x;
    if (o >= A.n_fl) return;
    const int32_t below = A.tab[(size_t)(5 - 1) * A.T + o];  // o - e_5 = o - z
    const bool fl = (uint32_t)below < (uint32_t)A.n_col;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        const R r = fl ? A.rho[(size_t)below * NC + k] : P.res_rho[1][k];
        R ps, u;
        psi_of(P, k, r, ps, u);
        A.rho[(size_t)o * NC + k] = r;
        A.psi[(size_t)o * NC + k] = ps;
        if (P.has_zc) A.U[(size_t)o * NC + k] = u;
    }
}

// Partial sums (sum u_c, count) of the fluid ids [lo, hi) of the plane below
// the outlet at time t, from this step's pulls; u_c = j_c / rho in FP64.
template <int NC, int ST>
__global__ void __launch_bounds__(kFlThreads)
    k_fl_conv_u(StepArgs<typename Store<ST>::R> P, FlArgs<typename Store<ST>::R> A, int lo, int hi,
                double* __restrict__ part) {
    using R = typename Store<ST>::R;
    const int e = lo + blockIdx.x * kFlThreads + threadIdx.x;
    double u = 0.0, cnt = 0.0;
    if (e < hi) {
        int32_t src[Q];
        R f[NC][Q];
        fl_pull<NC, ST>(P, A, e, src, f);
        double jc = 0.0, r = 0.0;
        for (int k = 0; k < NC; ++k)
            for (int i = 0; i < Q; ++i) {
                r += (double)f[k][i];
                jc += (double)f[k][i] * L::ec(i);
            }
        u = jc / r;
        cnt = 1.0;
    }
    __shared__ double sh[2][kFlThreads / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        u += __shfl_xor(u, off, 64);
        cnt += __shfl_xor(cnt, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        sh[0][threadIdx.x >> 6] = u;
        sh[1][threadIdx.x >> 6] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double su = 0.0, sc = 0.0;
        for (int w = 0; w < kFlThreads / 64; ++w) {
            su += sh[0][w];
            sc += sh[1][w];
        }
        part[2 * blockIdx.x] = su;
        part[2 * blockIdx.x + 1] = sc;
    }
}

// Ghost populations of the outlet ids after the step: for e_c(i) = -1,
//   g_i = (f_i(x, t) + U f_i(x - c, t + 1)) / (1 + U),
// x = o + e_i (the fluid node it streams into), f_i(x, t) = the value this
// step pulled (fin at o), f_i(x - c, t + 1) = the population streaming into
// the node below x (fout), U = max(0, mean u_c of the plane below).
template <int NC, int ST>
__global__ void __launch_bounds__(kFlThreads)
    k_fl_conv_ghost(StepArgs<typename Store<ST>::R> P, FlArgs<typename Store<ST>::R> A,
                    const double* __restrict__ part, int nblk) {
    using S = typename Store<ST>::S;
    using R = typename Store<ST>::R;
    const int o = A.n_col + blockIdx.x * kFlThreads + threadIdx.x;
    if (o >= A.n_fl) return;
    double su = 0.0, sc = 0.0;  // same order in every thread: one U for the plane
    for (int j = 0; j < nblk; ++j) {
        su += part[2 * j];
        sc += part[2 * j + 1];
    }
    double U = sc > 0.0 ? su / sc : 0.0;
    U = U > 0.0 ? U : 0.0;
    const size_t T = (size_t)A.T;
    const S* fin = reinterpret_cast<const S*>(P.fin);
    S* fout = reinterpret_cast<S*>(P.fout);
    const int32_t src = A.tab[(size_t)(5 - 1) * T + o];  // the node below o
    sfor<Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if constexpr (L::ec(i) == -1) {
            const int32_t x = A.tab[(size_t)(opp(i) - 1) * T + o];  // o + e_i
            if ((uint32_t)x >= (uint32_t)A.n_col) return;
            const int32_t xu = A.tab[(size_t)(5 - 1) * T + x];     // the node below x
            const bool xu_fl = (uint32_t)xu < (uint32_t)A.n_col;
            const bool src_fl = (uint32_t)src < (uint32_t)A.n_col;
            for (int k = 0; k < NC; ++k) {
                const R prev = (R)fin[(size_t)(k * Q + i) * T + o];
                R upw = prev;
                // f_i(x - c, t + 1): from xu - e_i = the node below o, or bounced back
                if (xu_fl) upw = src_fl ? (R)fout[(size_t)(k * Q + i) * T + src]
                                        : (R)fout[(size_t)(k * Q + opp(i)) * T + xu];
                fout[(size_t)(k * Q + i) * T + o] = (S)((prev + (R)U * upw) / ((R)1 + (R)U));
            }
        }
    });
}

// Flag (any thread may write it) if a fluid id has an unlisted neighbour.
__global__ void __launch_bounds__(kFlThreads)
    k_fl_check(const int32_t* __restrict__ tab, int n_fl, int T, int32_t* __restrict__ flag) {
    const int e = blockIdx.x * kFlThreads + threadIdx.x;
    if (e >= n_fl) return;
    bool bad = false;
    for (int i = 0; i < Q - 1; ++i) bad |= tab[(size_t)i * T + e] < 0;
    if (bad) *flag = 1;
}

template <class R>
FlArgs<R> fl_args(lbm_handle* h) {
    FlArgs<R> A;
    char* ws = h->ws;
    A.tab = reinterpret_cast<const int32_t*>(ws + h->lay.ftab);
    A.dmap = reinterpret_cast<const int32_t*>(ws + h->lay.fdmap);
    A.emap = reinterpret_cast<const int32_t*>(ws + h->lay.femap);
    A.rho = reinterpret_cast<R*>(ws + h->lay.frho);
    A.psi = reinterpret_cast<R*>(ws + h->lay.fpsi);
    A.U = reinterpret_cast<R*>(ws + h->lay.fU);
    A.n_col = h->n_col;
    A.n_fl = h->n_fl;
    A.n_sol = h->n_sol;
    A.n_r1 = h->n_r1;
    A.n_ext = h->n_ext;
    A.T = h->fl_T;
    return A;
}

inline int blocks(int n) { return (n + kFlThreads - 1) / kFlThreads; }

// psi of every listed node (passes 1 and 2)
template <int NC, int ST>
hipError_t launch_psi(lbm_handle* h, const StepArgs<typename Store<ST>::R>& a,
                      const FlArgs<typename Store<ST>::R>& A) {
    using R = typename Store<ST>::R;
    if (h->n_col > 0)
        hipLaunchKernelGGL((k_fl_rho<NC, ST>), dim3(blocks(h->n_col)), dim3(kFlThreads), 0, h->stream, a, A);
    if (h->n_fl > h->n_col)
        hipLaunchKernelGGL((k_fl_conv_rho<NC, R>), dim3(blocks(h->n_fl - h->n_col)), dim3(kFlThreads), 0, h->stream,
                           a, A);
    if (h->n_ext > h->n_fl)
        hipLaunchKernelGGL((k_fl_solid<NC, R>), dim3(blocks(h->n_ext - h->n_fl)), dim3(kFlThreads), 0, h->stream,
                           a, A);
    return hipGetLastError();
}

template <int NC, int ST>
hipError_t step_store(lbm_handle* h) {
    using R = typename Store<ST>::R;
    StepArgs<R> a;
    fill_args(h, a, nullptr);
    const FlArgs<R> A = fl_args<R>(h);
    hipError_t e = launch_psi<NC, ST>(h, a, A);
    if (e != hipSuccess || h->n_col == 0) return e;
    if (h->p.collision == LBM_MRT)
        hipLaunchKernelGGL((k_fl_step<NC, ST, COLL_MRT>), dim3(blocks(h->n_col)), dim3(kFlThreads), 0, h->stream, a,
                           A);
    else
        hipLaunchKernelGGL((k_fl_step<NC, ST, COLL_BGK>), dim3(blocks(h->n_col)), dim3(kFlThreads), 0, h->stream, a,
                           A);
    return hipGetLastError();
}

template <int NC, int ST>
hipError_t mom_store(lbm_handle* h, int comp, void* rho, void* u) {
    using R = typename Store<ST>::R;
    StepArgs<R> a;
    fill_args(h, a, nullptr);
    a.mom_comp = comp;
    a.mom_rho = reinterpret_cast<R*>(rho);
    a.mom_u = reinterpret_cast<R*>(u);
    const FlArgs<R> A = fl_args<R>(h);
    hipError_t e = launch_psi<NC, ST>(h, a, A);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_fl_mom<NC, ST>), dim3(blocks(h->N)), dim3(kFlThreads), 0, h->stream, a, A);
    return hipGetLastError();
}

template <int NC, int ST>
hipError_t init_store(lbm_handle* h, const void* rho0, const void* u0) {
    using R = typename Store<ST>::R;
    if (h->n_fl == 0) return hipSuccess;
    ResRho res;
    std::memcpy(res.r, h->res_active, sizeof(res.r));
    float* rout = is_dev(h->p.storage) ? reinterpret_cast<float*>(h->ws + h->lay.rA) : nullptr;
    hipLaunchKernelGGL((k_fl_init<NC, ST>), dim3(blocks(h->n_fl)), dim3(kFlThreads), 0, h->stream,
                       (const R*)rho0, (const R*)u0, fl_args<R>(h), h->ws + h->lay.fA, rout, h->N, res, h->NA, h->NB,
                       h->NCc);
    return hipGetLastError();
}

// Dispatch over components and storage (F64, F32, F32 with FP64 arithmetic,
// FP16 and BF16 deviations).
template <template <int, int> class Fn, class... Args>
hipError_t dispatch(lbm_handle* h, Args... args) {
    const int nc = h->p.n_comp;
    switch (h->p.storage) {
        case LBM_STORE_F64:
            return nc == 1 ? Fn<1, ST_F64>::run(h, args...) : Fn<2, ST_F64>::run(h, args...);
        case LBM_STORE_F32:
            return nc == 1 ? Fn<1, ST_F32>::run(h, args...) : Fn<2, ST_F32>::run(h, args...);
        case LBM_STORE_F32_F64:
            return nc == 1 ? Fn<1, ST_F32D>::run(h, args...) : Fn<2, ST_F32D>::run(h, args...);
        case LBM_STORE_F16DEV:
            return nc == 1 ? Fn<1, ST_F16>::run(h, args...) : Fn<2, ST_F16>::run(h, args...);
        case LBM_STORE_BF16DEV:
            return nc == 1 ? Fn<1, ST_BF16>::run(h, args...) : Fn<2, ST_BF16>::run(h, args...);
        default: return hipErrorInvalidValue;  // rejected at lbm_init
    }
}
template <int NC, int ST>
hipError_t conv_store(lbm_handle* h) {
    using R = typename Store<ST>::R;
    if (h->n_fl == h->n_col || h->conv_hi <= h->conv_lo) return hipSuccess;
    StepArgs<R> a;
    fill_args(h, a, nullptr);
    const FlArgs<R> A = fl_args<R>(h);
    double* part = reinterpret_cast<double*>(h->ws + h->lay.conv_part);
    const int nblk = blocks(h->conv_hi - h->conv_lo);
    hipLaunchKernelGGL((k_fl_conv_u<NC, ST>), dim3(nblk), dim3(kFlThreads), 0, h->stream, a, A, h->conv_lo,
                       h->conv_hi, part);
    hipLaunchKernelGGL((k_fl_conv_ghost<NC, ST>), dim3(blocks(h->n_fl - h->n_col)), dim3(kFlThreads), 0, h->stream,
                       a, A, (const double*)part, nblk);
    return hipGetLastError();
}

template <int NC, int ST>
struct ConvFn {
    static hipError_t run(lbm_handle* h) { return conv_store<NC, ST>(h); }
};
template <int NC, int ST>
struct StepFn {
    static hipError_t run(lbm_handle* h) { return step_store<NC, ST>(h); }
};
template <int NC, int ST>
struct MomFn {
    static hipError_t run(lbm_handle* h, int comp, void* rho, void* u) { return mom_store<NC, ST>(h, comp, rho, u); }
};
template <int NC, int ST>
struct InitFn {
    static hipError_t run(lbm_handle* h, const void* rho0, const void* u0) { return init_store<NC, ST>(h, rho0, u0); }
};

}  // namespace

int lbmi::fluid_build(lbm_handle* h) {
    const size_t N = (size_t)h->N;
    // which solid nodes have a fluid neighbour: from the neighbour words
    // (bit 0: the node is not fluid; bit i: x - e_i is solid or a reservoir;
    // NW_OWN_RES / NW_OWN_ID: the node is a reservoir node, of reservoir 1)
    std::vector<uint32_t> word;
    std::vector<int32_t> emap, dmap;
    try {
        word.resize(N);
        emap.assign(N, -1);
        dmap.reserve(N);
    } catch (...) {
        return LBM_ERR_OOM;
    }
    if (hipMemcpyAsync(word.data(), h->ws + h->lay.nbr, N * 4, hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess)
        return LBM_ERR_HIP;
    constexpr uint32_t ALLNB = ((1u << Q) - 1u) & ~1u;
    // fluid ids; [conv_lo, conv_hi): those of the plane below an outlet plane
    const size_t plane = (size_t)h->NA * h->NB;
    const size_t ci = h->conv_plane > 0 ? (size_t)(h->conv_plane - 1) : 0;
    h->conv_lo = h->conv_hi = 0;
    for (size_t n = 0; n < N; ++n) {
        if (h->conv_plane > 0 && n == ci * plane) h->conv_lo = (int)dmap.size();
        if (h->conv_plane > 0 && n == (ci + 1) * plane) h->conv_hi = (int)dmap.size();
        if (!(word[n] & 1u)) {
            emap[n] = (int32_t)dmap.size();
            dmap.push_back((int32_t)n);
        }
    }
    h->n_col = (int)dmap.size();
    // outlet nodes: pulled from like fluid, so their ids are below n_fl
    for (size_t n = 0; n < N; ++n)
        if (word[n] & NW_OWN_CONV) {
            emap[n] = (int32_t)dmap.size();
            dmap.push_back((int32_t)n);
        }
    h->n_fl = (int)dmap.size();
    for (size_t n = 0; n < N; ++n)
        if ((word[n] & 1u) && !(word[n] & (NW_OWN_RES | NW_OWN_CONV)) && (word[n] & ALLNB) != ALLNB) {
            emap[n] = (int32_t)dmap.size();
            dmap.push_back((int32_t)n);
        }
    h->n_sol = (int)dmap.size();
    // every reservoir node (whole planes): reservoir 0, then reservoir 1
    for (uint32_t id = 0; id < 2; ++id) {
        if (id == 1) h->n_r1 = (int)dmap.size();
        for (size_t n = 0; n < N; ++n)
            if ((word[n] & NW_OWN_RES) && ((word[n] & NW_OWN_ID) ? 1u : 0u) == id) {
                emap[n] = (int32_t)dmap.size();
                dmap.push_back((int32_t)n);
            }
    }
    h->n_ext = (int)dmap.size();
    h->fl_T = (int)((N + 63) / 64 * 64);
    // each node is listed at most once, so the ids fit the rows of T
    if (dmap.size() > N) return LBM_ERR_HIP;
    char* ws = h->ws;
    hipError_t e = hipMemcpyAsync(ws + h->lay.femap, emap.data(), N * 4, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess && h->n_ext > 0)
        e = hipMemcpyAsync(ws + h->lay.fdmap, dmap.data(), (size_t)h->n_ext * 4, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess && h->n_ext > 0) {
        hipLaunchKernelGGL(k_fl_table, dim3(blocks(h->n_ext)), dim3(kFlThreads), 0, h->stream,
                           reinterpret_cast<const int32_t*>(ws + h->lay.femap),
                           reinterpret_cast<const int32_t*>(ws + h->lay.fdmap),
                           reinterpret_cast<int32_t*>(ws + h->lay.ftab), h->n_ext, h->fl_T, h->NA, h->NB, h->NCc);
        e = hipGetLastError();
    }
    // every neighbour of a fluid node must be listed (fluid, solid next to
    // fluid, or reservoir), so that the step's pulls and gathers index only
    // listed ids; k_fl_check raises a flag (kept in the first word of the
    // density array, which the first step overwrites) where one is not
    int32_t* flag = reinterpret_cast<int32_t*>(ws + h->lay.frho);
    if (e == hipSuccess) e = hipMemsetAsync(flag, 0, 4, h->stream);
    if (e == hipSuccess && h->n_col > 0) {
        hipLaunchKernelGGL(k_fl_check, dim3(blocks(h->n_col)), dim3(kFlThreads), 0, h->stream,
                           reinterpret_cast<const int32_t*>(ws + h->lay.ftab), h->n_col, h->fl_T, flag);
        e = hipGetLastError();
    }
    int32_t bad = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&bad, flag, 4, hipMemcpyDeviceToHost, h->stream);
    // the host vectors must outlive the copies
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return LBM_ERR_HIP;
    return bad ? LBM_ERR_HIP : LBM_OK;  // neighbour words and listing disagree
}

hipError_t lbmi::fluid_init(lbm_handle* h, const void* rho0, const void* u0) {
    return dispatch<InitFn>(h, rho0, u0);
}

hipError_t lbmi::fluid_step(lbm_handle* h) { return dispatch<StepFn>(h); }

hipError_t lbmi::fluid_conv(lbm_handle* h) { return dispatch<ConvFn>(h); }

hipError_t lbmi::fluid_moments(lbm_handle* h, int comp, void* rho, void* u) {
    return dispatch<MomFn>(h, comp, rho, u);
}
