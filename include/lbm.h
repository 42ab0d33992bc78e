/*
 * C-ABI of the MI355X multiphase lattice-Boltzmann library (liblbm.so).
 *
 * One handle advances one lattice on one HIP stream with a fused kernel per
 * time step.  The step is the paper's Shan-Chen pseudopotential method for one
 * or two fluid components (Sec. 2.1-2.4):
 *   density and momentum moments                       (Eq. 4, Eq. 10)
 *   improved virtual density at solid nodes             (Eq. 17)
 *   EOS pseudopotential psi, U                          (Eq. 12)
 *   Shan-Chen / Zhang-Chen interaction force            (Eq. 11, Eq. 13)
 *   BGK or MRT collision with exact-difference forcing  (Eq. 3, Eq. 5)
 *   streaming with halfway bounce-back                  (Eq. 1, Eq. 2)
 *   open boundaries: reservoirs at fixed density        (Sec. 3.4.3)
 * and observes densities and velocities with the half-force correction
 * (Eq. 6), and in place the capillary pressure and saturation (Sec. 3.4.3).
 *
 * Conventions
 *   - Every function returns LBM_OK (0) or a negative lbm_error code; no
 *     exception or abort crosses the ABI.
 *   - Arrays are in (z, y, x) order, x fastest.  A D2Q9 lattice has nz = 1
 *     and its arrays are (y, x).
 *   - "host" pointers are ordinary CPU memory, read during the call;
 *     "device" pointers are HIP device memory owned by the caller.
 *   - A handle is bound to the stream given to lbm_init; calls on one handle
 *     are not thread-safe.  Work is enqueued asynchronously unless a function
 *     says it synchronises.
 *   - The compute type is double for LBM_STORE_F64 and LBM_STORE_F32_F64 and
 *     float otherwise; "compute-type" buffers below use it.
 */
#ifndef PAPER_2506_17713_LBM_H
#define PAPER_2506_17713_LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lbm_error {
    LBM_OK = 0,
    LBM_ERR_ARG = -1,         /* invalid argument or parameter combination   */
    LBM_ERR_UNSUPPORTED = -2, /* valid but not provided by this library       */
    LBM_ERR_HIP = -3,         /* a HIP runtime call or kernel launch failed   */
    LBM_ERR_NONFINITE = -4,   /* a check found a non-finite or negative rho   */
    LBM_ERR_SPACE = -5,       /* workspace smaller than lbm_workspace_size   */
    LBM_ERR_OOM = -6          /* host memory for the handle could not be had */
} lbm_error;

enum { LBM_D2Q9 = 0, LBM_D3Q19 = 1 };
/* Collision (Eq. 3): BGK or MRT with exact-difference forcing (Eq. 5), or
 * central moments (cascaded) with the consistent forcing of the same moments
 * (Eq. 7-8; D2Q9, one component; rates in mrt_s on the MRT rows evaluated at
 * the peculiar velocities e_i - u). */
enum { LBM_BGK = 0, LBM_MRT = 1, LBM_CLBM = 2 };
/* Population storage.  F64 / F32 store f_i and compute in the same type.
 * F32_F64 stores f_i in FP32 and computes in FP64: the memory and HBM
 * traffic of FP32 with the accuracy that FP32 rounding of the stored state
 * alone allows (long runs in FP32 arithmetic accumulate several times that).
 * F16DEV / BF16DEV store the relative deviation h_i = f_i / (w_i rho*) - 1 in
 * 16 bits plus the node's density rho* in FP32, and reconstruct
 * f_i = w_i rho* (1 + h_i) in FP32. */
enum { LBM_STORE_F64 = 0, LBM_STORE_F32 = 1, LBM_STORE_F16DEV = 2, LBM_STORE_BF16DEV = 3, LBM_STORE_F32_F64 = 4 };
/* Pseudopotential: Carnahan-Starling EOS (Eq. 12) or psi = rho. */
enum { LBM_PSI_CS = 0, LBM_PSI_DENSITY = 1 };
/* Improved virtual density (Eq. 17): rho_s = phi rho_ave or rho_ave - drho. */
enum { LBM_WET_PHI = 0, LBM_WET_DRHO = 1 };
/* Population layout in the workspace.
 * DENSE: every lattice node holds its populations (solid slots unused); the
 * fused kernel marches tiles of the lattice.
 * FLUID: only fluid nodes hold populations, listed in lattice order, with a
 * table of the 18 neighbour indices per fluid node and per solid node next to
 * fluid (porous media: at porosity 0.35 the dense rows carry about three
 * times the fluid bytes).  Same method and results as DENSE (pinned by the
 * parity tests); D3Q19 only, any storage, BGK or MRT, reservoirs and the
 * convective outlet (LBM_ERR_UNSUPPORTED otherwise), and lbm_grad is
 * LBM_ERR_UNSUPPORTED.  The state of lbm_get_state / lbm_set_state is the
 * fluid-node populations (lbm_state_bytes). */
enum { LBM_LAYOUT_DENSE = 0, LBM_LAYOUT_FLUID = 1 };

#define LBM_MAX_COMP 2
#define LBM_MAX_Q 19

typedef struct lbm_params {
    int32_t lattice;            /* LBM_D2Q9 or LBM_D3Q19                       */
    int32_t nx, ny, nz;         /* lattice extent; nz = 1 for D2Q9; at most
                                   2^31 - 1 nodes and nx*ny < 2^29 (3-D)       */
    int32_t n_comp;             /* 1 or 2 fluid components                     */
    int32_t collision;          /* LBM_BGK, LBM_MRT or LBM_CLBM                */
    int32_t storage;            /* LBM_STORE_*                                 */
    int32_t psi_kind[2];        /* LBM_PSI_* per component                     */
    int32_t wet_mode[2];        /* LBM_WET_* per component                     */
    int32_t common_velocity;    /* two components: 1 = common velocity u' =
                                   sum_k(j^k/tau_k) / sum_k(rho^k/tau_k) in the
                                   equilibria; 0 = each component's j^k/rho^k  */
    int32_t check_every;        /* > 0: run the lbm_stats reduction every
                                   check_every steps inside lbm_step and latch
                                   LBM_ERR_NONFINITE; 0: checks on demand only  */
    int32_t reserved[4];        /* must be zero                                */
    double tau[2];              /* BGK relaxation time per component (> 0.5)   */
    double mrt_s[2][19];        /* MRT relaxation rate of each moment row, rows
                                   in the Lallemand-Luo (D2Q9) / d'Humieres
                                   (D3Q19) order                               */
    double eos_a[2], eos_b[2], eos_R[2];  /* Carnahan-Starling a, b, R         */
    double eos_T[2];            /* absolute temperature                         */
    double alpha[2];            /* EOS pressure scale alpha^k (Eq. 12)          */
    double A[2];                /* Zhang-Chen weight A_kk (Eq. 13)              */
    double g[2][2];             /* interaction strengths g_kk' (g_kk < 0 with
                                   the EOS pseudopotential)                     */
    double body_accel[3];       /* body acceleration (x, y, z): F^k += rho^k a  */
    double wet[2];              /* uniform phi or drho when no per-node array   */
    double rho_min[2], rho_max[2]; /* virtual-density limiter bounds            */
    double kappa[2];            /* surface-tension adjustment kappa^k (Sec. 2.3,
                                   Eq. 14-16): D2Q9 MRT adds the moment source
                                   C built from the pressure-tensor term Q, and
                                   the surface tension falls about as 1 - kappa
                                   with the coexistence densities unchanged.
                                   Q takes the factor g_kk, which the printed
                                   Eq. 16 leaves out.  0 = off; nonzero with
                                   D3Q19 or BGK: LBM_ERR_UNSUPPORTED           */
    double res_rho[2][2];       /* res_rho[r][k]: fixed density of component k
                                   in reservoir r (mask value 2 + r); > 0 for
                                   every reservoir the mask uses               */
    int32_t window[2];          /* planes window[0] <= c < window[1] of the
                                   slowest axis (z; y in 2-D) over which
                                   lbm_stats measures the capillary pressure
                                   and wetting saturation; window[1] <=
                                   window[0]: every plane                      */
    int32_t layout;             /* LBM_LAYOUT_DENSE or LBM_LAYOUT_FLUID         */
    int32_t reserved2;          /* must be zero                                */
} lbm_params;

typedef struct lbm_stats_t {
    int64_t step;               /* time steps taken since lbm_init              */
    double mass[2];             /* sum of rho^k over fluid nodes                */
    double momentum[3];         /* sum of the mixture momentum (Eq. 6)          */
    double residual;            /* sum|u_x - u_x(prev)| / sum|u_x| against the
                                   previous reduction (1.0 on the first one)    */
    double saturation;          /* fraction of fluid nodes classified non-wetting:
                                   rho^0 >= rho^1 (two components) or
                                   rho < (rho_min + rho_max)/2 (one component)  */
    double mean_ux;             /* mean mixture u_x over fluid nodes            */
    int64_t n_fluid;            /* number of fluid nodes                        */
    int32_t nonfinite;          /* count of fluid nodes with non-finite values  */
    int32_t negative;           /* count of fluid nodes with rho^k < 0          */
    /* In-situ capillary pressure and saturation (Sec. 3.4.3) over the fluid
     * nodes of the parameter window, each classed as for `saturation`;
     * pressure p = c_s^2 sum_k rho^k + (1/2) sum_kk' g_kk' psi^k psi^k'
     * (alpha p_EOS for one component with the EOS pseudopotential). */
    double p_nonwetting;        /* mean p over the non-wetting nodes (0: none)  */
    double p_wetting;           /* mean p over the wetting nodes (0: none)      */
    double capillary_pressure;  /* p_nonwetting - p_wetting                     */
    double s_wetting;           /* wetting nodes / fluid nodes of the window    */
} lbm_stats_t;

typedef struct lbm_handle lbm_handle;

/* Device bytes lbm_init needs in its workspace for these parameters: two
 * population buffers (ping-pong), the per-node neighbour words, the wetting
 * field, moment scratch and reduction partials; with LBM_LAYOUT_FLUID also
 * the neighbour table and the per-node density and pseudopotential arrays
 * (sized for the worst case, every node fluid).  Pure function.
 * Errors: LBM_ERR_ARG for an invalid parameter set. */
int lbm_workspace_size(const lbm_params* p, size_t* bytes_out);

/* Create a handle and set the populations to the equilibrium of rho0/u0
 * (Eq. 3 with the moments given; the initial state of the droplet, slab and
 * pore-filling runs of Sec. 3).
 *   p          parameters, copied.
 *   mask       host uint8[N]: 0 = fluid, 1 = solid (walls, grains; halfway
 *              bounce-back), 2 / 3 = reservoir 0 / 1, 4 = convective outlet.  A reservoir is an open
 *              boundary (Sec. 3.4.3: constant-pressure inlet and outlet) held
 *              at the densities p->res_rho[r] and at rest: a population that
 *              would stream in from it is 2 w_i rho_res - f*_opp(i)(x) (anti-
 *              bounce-back, which fixes the density halfway between the
 *              reservoir and x), and its psi(rho_res) enters the force and
 *              virtual densities of its neighbours.  Reservoir nodes must fill
 *              whole planes of the slowest axis (z; y in 2-D), one reservoir
 *              per plane, and no fluid node may touch reservoir planes on
 *              both sides (LBM_ERR_ARG otherwise).
 *              A convective outlet (Sec. 3.4.2) is one whole plane with fluid
 *              in the plane below it and none above: a population that
 *              streams down into the fluid from it follows the convective
 *              equation d f/dt + U d f/dc = 0, (f(t) + U f_below(t+1)) /
 *              (1 + U), with U = max(0, mean j_c / rho) over the fluid of the
 *              plane below at time t; its density in the force gather is
 *              that of the node below it (res_rho[1] where that is solid).
 *              Not with 16-bit storage (LBM_ERR_UNSUPPORTED).
 *   rho0       host double[n_comp][N], initial density per component.
 *   u0         host double[3][N] initial equilibrium velocity j/rho (x, y, z),
 *              or NULL for rest.  The velocity of Eq. 6 reported by
 *              lbm_moments adds F/(2 rho) to it.
 *   wet        host double[n_comp][N] per-node phi / drho (used at solid
 *              nodes), or NULL to use p->wet uniformly.
 *   workspace  device buffer of ws_bytes >= lbm_workspace_size(p); owned by
 *              the caller and must outlive the handle.
 *   stream     hipStream_t on which all work of this handle is enqueued
 *              (NULL = the null stream).
 * Synchronises the stream before returning.
 * Errors: LBM_ERR_ARG (bad parameters, NaN or negative rho0), LBM_ERR_SPACE,
 * LBM_ERR_UNSUPPORTED, LBM_ERR_OOM, LBM_ERR_HIP. */
int lbm_init(const lbm_params* p, const uint8_t* mask, const double* rho0, const double* u0,
             const double* wet, void* workspace, size_t ws_bytes, void* stream,
             lbm_handle** out);

/* Enqueue nsteps fused time steps (Eq. 1-17 in order) on the handle's stream.
 * Asynchronous.  With check_every > 0 a reduction runs every check_every
 * steps; a non-finite or negative density is reported by the next lbm_stats
 * or lbm_sync.  Errors: LBM_ERR_ARG (nsteps < 0), LBM_ERR_HIP. */
int lbm_step(lbm_handle* h, int64_t nsteps);

/* Write the current density and velocity (Eq. 6, u = (j + F/2) / rho) into
 * caller-owned device buffers of the compute type:
 *   comp >= 0: rho_dev[N] = rho^comp, u_dev[3][N] = (j^comp + F^comp/2)/rho^comp
 *   comp = -1: rho_dev[N] = sum_k rho^k, u_dev = sum_k(j^k + F^k/2)/sum_k rho^k
 * Solid nodes get 0.  Either pointer may be NULL.  Asynchronous.
 * Errors: LBM_ERR_ARG, LBM_ERR_HIP. */
int lbm_moments(lbm_handle* h, int comp, void* rho_dev, void* u_dev);

/* Reduce the current state (FP64 accumulation, fixed order: bitwise
 * reproducible) and copy the result to *out: the masses of Eq. 4/10, the
 * mixture momentum and mean u_x of Eq. 6 (Darcy permeability, Sec. 3.4.1),
 * the saturation S_w of Sec. 3.4.3 and the steady-state residual.
 * Synchronises the stream.
 * Returns LBM_ERR_NONFINITE if this or a latched periodic check saw a
 * non-finite or negative density (the latch is cleared). */
int lbm_stats(lbm_handle* h, lbm_stats_t* out);

/* Synchronise the stream; report a latched check failure or HIP error. */
int lbm_sync(lbm_handle* h);

/* New fixed densities rho[n_comp] (host) of reservoir r (0 or 1) from the
 * next step on: the inlet or outlet pressure of a drainage or imbibition
 * run, raised in stages to trace a capillary pressure - saturation curve
 * (Sec. 3.4.3).  The populations that stream in during the next lbm_step
 * and later take the new density; the current state (what lbm_moments and
 * lbm_stats see before that step) keeps the old one.  Errors: LBM_ERR_ARG
 * (r out of range, a density not finite and positive). */
int lbm_set_reservoir(lbm_handle* h, int r, const double* rho);

/* Restart from f = f^eq(rho0, u0) (Eq. 3 with the moments given), as
 * lbm_init does, but from device arrays: for callers whose initial fields
 * are computed on the GPU (a learned warm start).  rho0_dev [n_comp][N] and
 * u0_dev [3][N] (NULL: rest) are device arrays of the compute type, node order as in lbm_init; values at
 * solid nodes are ignored.  Unlike lbm_init the values are not validated: a
 * non-finite or negative density is reported by the next check.  The step
 * counter and the residual history restart; mask, parameters and wetting
 * field are kept.  Synchronises the stream.  Errors: LBM_ERR_ARG, LBM_ERR_HIP. */
int lbm_reset(lbm_handle* h, const void* rho0_dev, const void* u0_dev);

/* Bytes of the raw population state (layout private to this library). */
int lbm_state_bytes(const lbm_handle* h, size_t* bytes_out);
/* Copy the raw state to / from a device buffer of lbm_state_bytes bytes
 * (checkpoint and resume).  Asynchronous on the handle's stream. */
int lbm_get_state(lbm_handle* h, void* dev_dst);
int lbm_set_state(lbm_handle* h, const void* dev_src);

/* ------------------------------------------------------------------------
 * Gradients by the hand-written adjoint of the fused step (reverse mode).
 * The paper differentiates its solver end to end with JAX (Sec. 4); this is
 * the same derivative, computed by an explicit adjoint of every step (Eq. 1-17
 * in reverse) with checkpointing every ckpt_every steps.
 *
 * Observables of the density rho(x) at the final step:
 *   LBM_OBS_SATURATION  L = (1/N_fluid) sum_fluid sigma((rho_mid - rho) / delta),
 *                       a smooth fraction of fluid nodes below rho_mid (the
 *                       non-wetting vapour); sigma is the logistic function.
 *                       (Sec. 3.4.3 segments by threshold; the step function
 *                       has no derivative, the logistic one does.)
 *   LBM_OBS_DRHO        L = sum_x dL_drho[x] rho(x) with a caller-given device
 *                       array dL_drho[N] of the compute type (any objective
 *                       linearised in the final density).
 * Supported for one component with LBM_STORE_F32 or LBM_STORE_F64, BGK or
 * MRT, no surface-tension source and no reservoirs; other configurations
 * (two components, 16-bit storage, LBM_STORE_F32_F64, kappa != 0, LBM_CLBM,
 * reservoir nodes) return LBM_ERR_UNSUPPORTED.
 * ------------------------------------------------------------------------ */
enum { LBM_OBS_SATURATION = 0, LBM_OBS_DRHO = 1 };

typedef struct lbm_grad_req {
    int32_t observable;         /* LBM_OBS_*                                    */
    int32_t nsteps;             /* forward horizon (>= 1)                       */
    int32_t ckpt_every;         /* checkpoint interval K (>= 1)                 */
    int32_t reserved;           /* must be zero                                 */
    double rho_mid, delta;      /* LBM_OBS_SATURATION parameters (delta > 0)    */
    const void* dL_drho;        /* LBM_OBS_DRHO: device array [N]               */
    void* ws;                   /* device workspace, 256-byte aligned, owned by
                                   the caller: checkpoints, one segment of states
                                   and the adjoint fields                       */
    size_t ws_bytes;
} lbm_grad_req;

/* Device bytes lbm_grad needs in r->ws for this handle and request:
 * ceil(nsteps/K) checkpoints plus K recomputed states (each q*N values of the
 * compute type) and about 2q + 15 values per node of adjoint fields.
 * Errors: LBM_ERR_ARG, LBM_ERR_UNSUPPORTED. */
int lbm_grad_workspace_size(const lbm_handle* h, const lbm_grad_req* r, size_t* bytes_out);

/* Starting from the handle's current state, run nsteps forward steps (the
 * handle ends advanced by nsteps, as after lbm_step), evaluate L and
 * back-propagate.  Outputs:
 *   L_out      host: value of the observable (may be NULL)
 *   dwet_dev   device double[N]: dL / d(wetting parameter) per node (phi or
 *              drho by wet_mode), non-zero only at solid nodes next to fluid
 *              whose virtual density is not at a limiter bound
 *   dT_out     host: dL / d eos_T[0] (absolute temperature; may be NULL)
 * Synchronises the stream.  Errors: LBM_ERR_ARG, LBM_ERR_SPACE,
 * LBM_ERR_UNSUPPORTED, LBM_ERR_HIP. */
int lbm_grad(lbm_handle* h, const lbm_grad_req* r, double* L_out, double* dwet_dev, double* dT_out);

/* Release the handle (not the caller's workspace).  NULL is ignored. */
void lbm_free(lbm_handle* h);

/* Static description of an error code. */
const char* lbm_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* PAPER_2506_17713_LBM_H */
