/*
 * mgso.h -- C ABI of the moving-grid split-operator library (gfx950 / MI355X).
 *
 * The method: Choi & Vanicek, "A time-reversible integrator for the time-dependent
 * Schroedinger equation on an adaptive grid" (arXiv:1909.06412).  Equation numbers
 * count the paper's displayed equations in order of appearance.
 *
 * Problem statement followed by this interface (Sec. II):
 *   H = T(p) + V(q) with T = p^T m^-1 p / 2 and a diagonal mass matrix (Eqs. (2)-(3));
 *   the wavefunction lives on a D-dimensional tensor-product grid
 *   q_l^J = q_ctr,l + (j_l - N_l/2) dq_l, p_l^K = p_ctr,l + (k_l - N_l/2) dp_l,
 *   dq_l dp_l = 2 pi hbar / N_l (Eqs. (9)-(10));
 *   one step is a symmetric composition (Eq. (6)) of TVT or VTV stages (Eq. (5)) of the
 *   adaptive substeps U_V,adpt and U_T,adpt (Sec. II.G, Eqs. (45)-(47), (51)-(55)), which
 *   move the grid centres with the Ehrenfest moments <dV/dq> and <p>.
 *
 * Conventions shared by every entry point
 *   - Arrays over the grid are C-ordered: the last axis is contiguous.
 *   - Wavefunction values exchanged with the caller are physical psi(q^J) as
 *     interleaved (re, im) FP64 pairs, 2*N doubles (the paper scales back to physical
 *     values at the end, Sec. II.D).  On the device the library keeps
 *     c_J = psi(q^J) sqrt(prod_l dq_l) in the context's precision.
 *   - Host pointers are borrowed for the duration of the call and copied.
 *   - Device buffers bound with mg_bind_buffers are borrowed until mg_destroy; the
 *     library never frees them.  Unbound buffers are allocated by the library.
 *   - Every call returns an mg_status; nothing throws across the ABI.  mg_last_error
 *     gives a message for the last failing call on a context.
 *   - All device work is enqueued on the context's HIP stream (the one passed at
 *     creation, or the null stream).  mg_step, mg_observables, mg_get_state and
 *     mg_adjoint synchronise that stream before returning.
 *   - Grid centres, moments and composition coefficients are FP64 in every precision.
 *   - After MG_EUNSTABLE the state is invalid until the next set_* call.
 */
#ifndef MGSO_H
#define MGSO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MG_MAX_DIM 8          /* largest D (the paper's 8-D Henon-Heiles model) */
#define MG_MAX_AXIS 4096      /* largest N_l; each N_l is even and 2^a 3^b 5^c    */

typedef enum {
  MG_OK = 0,
  MG_EINVAL = -1,     /* bad argument: shape, size, kind, parameter count, order */
  MG_ENOMEM = -2,     /* device or host allocation failed                        */
  MG_EDEVICE = -3,    /* a HIP call failed                                       */
  MG_EUNSTABLE = -4,  /* non-finite moments or centres, or a substep moved the
                         grid by more than half its span (Sec. II.H: the grid
                         centres follow Stoermer-Verlet and diverge beyond the
                         bound of Eq. (57))                                       */
  MG_ESTATE = -5      /* call out of order (e.g. step before a state is set)      */
} mg_status;

typedef enum { MG_C128 = 0, MG_C64 = 1 } mg_precision;   /* storage + FFT precision */

typedef enum {
  MG_POT_FREE = 0,           /* V = 0                                     params: none  */
  MG_POT_HARMONIC = 1,       /* V = 1/2 sum_l k_l (q_l - s_l)^2           params: k[D], s[D] */
  MG_POT_MORSE_REP = 2,      /* V = De (1 - exp(-a (q0 - re)))^2 + A exp(-b (q1 - c q0))
                                (D = 2; D = 1 keeps the Morse term)       params: De,a,re,A,b,c
                                The modified Secrest-Johnson surface of Sec. III.B, Eq. (61),
                                is De = D, a = beta, re = 0, A = 1, b = alpha, c = 1.      */
  MG_POT_HENON_HEILES = 3,   /* Sec. III.C: kappa/2 sum q_l^2 + lam sum (q_l^2 q_{l+1}
                                - q_{l+1}^3 / 3)                          params: kappa, lam */
  MG_POT_QUADRATIC = 4       /* V = 1/2 (q - s)^T K (q - s), K symmetric (Sec. III.A,
                                Eq. (60)); D <= 4                         params: K[D*D], s[D] */
} mg_pot;

typedef enum { MG_TVT = 0, MG_VTV = 1 } mg_split;        /* Eq. (5) and the remark after Eq. (6) */

typedef enum {
  MG_COMP_STRANG = 0,        /* a single TVT (VTV) stage, order 2                        */
  MG_COMP_SUZUKI = 1,        /* Suzuki's fractal, stages 5^(order/2-1)                   */
  MG_COMP_TRIPLE_JUMP = 2,   /* Yoshida's triple jump, stages 3^(order/2-1)              */
  MG_COMP_USER = 3           /* caller-supplied palindromic gammas summing to one        */
} mg_comp;

/* Options for mg_set_option. */
typedef enum {
  MG_OPT_ENGINE = 1,         /* sweep kernels of a single grid: 0 = automatic (the radix-16
                                register kernels when D >= 3 and every axis has 16
                                points, with the three-pass plan for 16^8 grids;
                                else the Stockham LDS sweeps), 1 = the Stockham
                                LDS sweeps for every grid, 2 = the radix-16 kernels
                                without the three-pass plan                               */
  MG_OPT_GRAPH = 2,          /* 1 = capture the launches of mg_step / mg_batch_step once
                                per (dt, nsteps) as a hipGraph and replay it; any set_*
                                or option call re-captures on the next step              */
  MG_OPT_PROFILE = 3,        /* 1 = time every sweep kernel with HIP events               */
  MG_OPT_RENORMALIZE = 4,    /* 1 = rescale to the FP64 norm after every potential substep
                                (a deviation from the paper, off by default)              */
  MG_OPT_GRID = 5            /* grid scheme (Sec. II.F-G): 0 = the time-reversible moving
                                grid (default); 1 = fixed grid (centres held); 2 = naive
                                adaptive grid: each step on the frozen grid, then re-centred
                                on <q>, <p> (Eqs. (29)-(34); not time reversible).  Batches
                                offer 0 and 1; the adjoint needs 0                        */
} mg_option;

typedef struct mg_ctx mg_ctx;

/* ---------------------------------------------------------------------------
 * Creation and buffers
 * ------------------------------------------------------------------------- */

/* Create a context for one wavepacket on a D-dimensional grid (Sec. II.B).
 *   D           1..MG_MAX_DIM
 *   N[D]        points per axis, each even, 2..MG_MAX_AXIS, of the form 2^a 3^b 5^c
 *   dq[D]       position spacings (> 0); momentum spacings are 2 pi hbar / (N_l dq_l)
 *   inv_mass[D] diagonal of m^-1 (Eq. (3))
 *   hbar        > 0
 *   prec        MG_C128 or MG_C64
 *   hip_stream  a hipStream_t, or NULL for the null stream
 * Errors: MG_EINVAL on any bad argument, MG_EDEVICE / MG_ENOMEM from HIP. */
mg_status mg_create(int D, const int32_t* N, const double* dq, const double* inv_mass,
                    double hbar, mg_precision prec, void* hip_stream, mg_ctx** out);
void mg_destroy(mg_ctx* ctx);

/* Bytes of the wavefunction buffer (N complex values in the context's precision) and
 * of the workspace (a second buffer of the same size, used by observables/regrid). */
size_t mg_state_bytes(const mg_ctx* ctx);
size_t mg_workspace_bytes(const mg_ctx* ctx);

/* Bind caller-owned device buffers (e.g. from PyTorch).  psi_dev must hold
 * mg_state_bytes, work_dev mg_workspace_bytes (or NULL: allocated on first use);
 * both 256-byte aligned.  Binding discards the current state (MG_ESTATE until set). */
mg_status mg_bind_buffers(mg_ctx* ctx, void* psi_dev, void* work_dev);

/* Device pointer of the wavefunction (c_J layout above); NULL before allocation. */
void* mg_state_ptr(mg_ctx* ctx);

/* ---------------------------------------------------------------------------
 * State
 * ------------------------------------------------------------------------- */

/* Sample prod_l (pi sigma_l^2)^(-1/4) exp[-(q_l-q0_l)^2/(2 sigma_l^2) + i p0_l (q_l-q0_l)/hbar]
 * (the Gaussian of Sec. III.B, Eq. (62), one factor per axis) on the grid centred at
 * q_ctr = q0 with p_ctr = p0 (the analytic expectation values; Sec. II.E centres the
 * grid on them).  Computed in FP64 on the device.  t is reset to 0. */
mg_status mg_set_gaussian(mg_ctx* ctx, const double* q0, const double* p0, const double* sigma);

/* Replace the state: psi_phys[2N] physical values at q^J on the grid centred at
 * q_ctr[D], momentum-grid centre p_ctr[D], time t. */
mg_status mg_set_state(mg_ctx* ctx, const double* psi_phys, const double* q_ctr,
                       const double* p_ctr, double t);

/* Read the state back (any output pointer may be NULL).  Synchronises. */
mg_status mg_get_state(mg_ctx* ctx, double* psi_phys, double* q_ctr, double* p_ctr, double* t);

/* ---------------------------------------------------------------------------
 * Model and scheme
 * ------------------------------------------------------------------------- */

/* Set V (see mg_pot for the parameter layout).  MG_EINVAL on a wrong count or D. */
mg_status mg_set_potential(mg_ctx* ctx, mg_pot kind, const double* params, int nparams);

/* Set the splitting and the composition (Eq. (6)).  order is even, 2..10 for the
 * built-in families; for MG_COMP_USER gammas[nstages] must be palindromic and sum
 * to one within 1e-12 (MG_EINVAL otherwise). */
mg_status mg_set_scheme(mg_ctx* ctx, mg_split split, mg_comp comp, int order,
                        const double* gammas, int nstages);

/* ---------------------------------------------------------------------------
 * Propagation and observables
 * ------------------------------------------------------------------------- */

/* Advance nsteps composition steps of size dt (dt < 0 propagates backward; the
 * method is time-reversible, Sec. II.G).  Adjacent kinetic (TVT) or potential (VTV)
 * halves of neighbouring stages are merged, which is exact: both substeps are exact
 * flows of the same separable Hamiltonian piece.  Synchronises; returns MG_EUNSTABLE
 * if any substep reported non-finite moments or an over-large shift. */
mg_status mg_step(mg_ctx* ctx, double dt, int64_t nsteps);

/* out[4 + 4D]: norm (Eq. (28)), <q>[D], <p>[D], q_ctr[D], p_ctr[D], Ekin, Epot, t.
 * <p> and Ekin are evaluated on the momentum grid, <q> and Epot on the position grid,
 * each normalised by the norm.  Synchronises. */
mg_status mg_observables(mg_ctx* ctx, double* out);

/* Trigonometric interpolation of the state onto the grid centred at new_q_ctr (the
 * same p_ctr): f~(q_new, p_ctr) f(q_ctr, p_ctr) psi with the transforms of Sec. II.C. */
mg_status mg_regrid(mg_ctx* ctx, const double* new_q_ctr);

/* Options (mg_option).  MG_EINVAL for unknown options or values. */
mg_status mg_set_option(mg_ctx* ctx, int option, int64_t value);

/* Kernel timing collected under MG_OPT_PROFILE since the last reset:
 * for the sweep kernel class with the largest total time, its launch count, total
 * milliseconds and algorithmic bytes per launch (2 x N x bytes per complex; 1 x for
 * a moments-only sweep, which stores nothing).
 * reset != 0 clears the counters after reading. */
mg_status mg_profile_read(mg_ctx* ctx, int64_t* launches, double* total_ms,
                          double* bytes_per_launch, int reset);
/* The kernel class that mg_profile_read reports (read it before a reset): sweep
 * index (0 = the sweep over the innermost axes), dir (0 forward, 1 inverse), the
 * epilogue flags of that sweep (1: momentum moments, 4: potential substep) and the
 * number of axes the sweep transforms together, and its mode: 0 an ordinary sweep,
 * 1 the moments-only forward sweep and 2 the round-trip inverse sweep (forward DFT,
 * kinetic factor, inverse DFT) that 16-point grids use for the outermost sweep of a
 * kinetic substep when it transforms one axis, 3 a pass of the three-pass 16^8
 * plan (sweep 1: the pass over axes 3, 0 and the high digit of axis 2; sweep 2: axes
 * 4, 1 and the low digit; group_axes 3), 4 its moments-only forward pass.  All
 * outputs -1 when nothing has been profiled.  Any output pointer may be NULL. */
mg_status mg_profile_class(const mg_ctx* ctx, int* sweep, int* dir, int* epi, int* group_axes,
                           int* mode);

/* Autocorrelation <psi_0|psi_t> (Sec. III.C): psi_0 is the Gaussian of
 * mg_set_gaussian with these parameters (q0, p0, sigma each [D]), evaluated
 * analytically on the current (moved) grid; the inner product is Eq. (28).
 * out[2] = (Re, Im), reduced in FP64.  Synchronises. */
mg_status mg_autocorrelation(mg_ctx* ctx, const double* q0, const double* p0, const double* sigma,
                             double* out);
/* Spectrum from an autocorrelation series (Sec. III.C, Fig. 9): for each energy E_k,
 * out[k] = Re integral_0^T <psi_0|psi_t> exp(-(t/t_damp)^2) exp(i E_k t / hbar) dt by the
 * trapezoidal rule over the n samples times[n], acf[2n] (Re, Im interleaved).  Host
 * arithmetic on the caller's arrays; no device work. */
mg_status mg_spectrum(const double* times, const double* acf, int n, const double* energies, int ne,
                      double t_damp, double hbar, double* out);

/* Adjoint of a whole propagation (reverse sweep over the substeps, with the state
 * checkpointed every K steps and recomputed forward inside each block).
 * Objective on the final grid: J = sum_J W(q^J) |c_J|^2 with
 *   W = 1 / (1 + exp(-(R_d - R)/w)), R = q1 - c q0 for D = 2 (c from the potential,
 *   or 0.5 for non-Morse kinds), or R = q0 for D = 1;  window = {R_d, w}.
 * The gradient is taken with respect to the potential parameters named by
 * param_ids (indices into the mg_set_potential parameter list; supported for
 * MG_POT_MORSE_REP ids 3 (A) and 4 (b), MG_POT_HARMONIC ids 0..D-1 (k_l)).
 * The propagation itself is left applied (the state ends at t + nsteps dt).
 * J_out[1], grad_out[nparams].  Synchronises.  MG_EINVAL for unsupported ids. */
mg_status mg_adjoint(mg_ctx* ctx, double dt, int64_t nsteps, int K, const double* window,
                     const int* param_ids, int nparams, double* J_out, double* grad_out);

/* ---------------------------------------------------------------------------
 * Batches: many independent wavepackets with their own grids, one launch.
 * ------------------------------------------------------------------------- */
typedef struct mg_batch mg_batch;

/* B packets, each D-dimensional with its own N[b*D + l] and dq[b*D + l]; shared
 * inv_mass[D], hbar, precision and stream.  The packets are stored back to back. */
mg_status mg_batch_create(int B, int D, const int32_t* N, const double* dq,
                          const double* inv_mass, double hbar, mg_precision prec,
                          void* hip_stream, mg_batch** out);
void mg_batch_destroy(mg_batch* b);
/* Gaussians per packet: q0, p0, sigma each [B*D]. */
mg_status mg_batch_set_gaussian(mg_batch* b, const double* q0, const double* p0,
                                const double* sigma);
mg_status mg_batch_set_potential(mg_batch* b, mg_pot kind, const double* params, int nparams);
mg_status mg_batch_set_scheme(mg_batch* b, mg_split split, mg_comp comp, int order,
                              const double* gammas, int nstages);
/* All packets advance nsteps of dt in ONE persistent kernel launch.  Synchronises. */
mg_status mg_batch_step(mg_batch* b, double dt, int64_t nsteps);
/* out[B * (4 + 4D)], per packet in the layout of mg_observables.  Synchronises. */
mg_status mg_batch_observables(mg_batch* b, double* out);
/* Packet idx: physical values (2 * N_idx doubles) and centres.  Synchronises. */
mg_status mg_batch_get_state(mg_batch* b, int idx, double* psi_phys, double* q_ctr,
                             double* p_ctr, double* t);
mg_status mg_batch_set_state(mg_batch* b, int idx, const double* psi_phys,
                             const double* q_ctr, const double* p_ctr, double t);
/* Batched adjoint with the objective of mg_adjoint per packet: J_out[B],
 * grad_out[B * nparams]. */
mg_status mg_batch_adjoint(mg_batch* b, double dt, int64_t nsteps, int K,
                           const double* window, const int* param_ids, int nparams,
                           double* J_out, double* grad_out);
mg_status mg_batch_set_option(mg_batch* b, int option, int64_t value);

/* Launch shapes of the batch step kernel: MG_BATCH_CONFIGS pairs (threads per
 * workgroup, points a workgroup keeps in LDS as one tile); index 0 is the default.
 * A packet of at most `tile` points stays in LDS for a whole mg_batch_step call;
 * larger packets sweep through global memory tile by tile.  Shapes 3 and 4 run
 * the tile transforms out of place between two LDS buffers (a smaller tile, fewer
 * registers and barriers per pass, composite radices up to 16).  Shape 5 is not
 * persistent: every sweep of every packet is one launch over 4096-point tiles and
 * each moment reduction one launch with a workgroup per packet, so large packets
 * spread over the whole device.  mg_batch_config reads pair `index` for the
 * batch's precision (MG_EINVAL out of range). */
#define MG_BATCH_CONFIGS 6
mg_status mg_batch_config(const mg_batch* b, int index, int* threads, int* tile);
/* Use launch shape `index` for the following mg_batch_step calls (builds that
 * shape's per-packet plans on first use).  The batched adjoint keeps index 0. */
mg_status mg_batch_set_config(mg_batch* b, int index);
/* The batch's own autotuner: times probe_steps steps of dt with every launch shape
 * on the batch's current state (HIP events around the launch), restores that state
 * exactly, and keeps the fastest shape.  ms_per_step[MG_BATCH_CONFIGS] (may be
 * NULL) receives the measured times, chosen the index kept.  Synchronises;
 * allocates a copy of the batch state for the duration of the call. */
mg_status mg_batch_autotune(mg_batch* b, double dt, int64_t probe_steps, double* ms_per_step, int* chosen);
/* Total points (sum over packets). */
int64_t mg_batch_points(const mg_batch* b);

/* ---------------------------------------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops or harnesses that forbid hipMalloc): the propagation of mg_step
 * (moving grid, Sec. II.G) as one call that allocates nothing on the device.
 *
 * psi_dev: the caller's device buffer of prod(N) complex values in `prec`
 *   (interleaved float2 / double2, C-ordered), holding c_J = psi(q^J) sqrt(prod dq)
 *   -- the layout of mg_state_ptr's buffer; 256-byte aligned; read and overwritten
 *   in place with the state after nsteps steps of dt.
 * q_ctr, p_ctr: host arrays [D], the grid centres on entry, overwritten with the
 *   centres at the end.  Grid, masses, potential (as mg_set_potential) and scheme
 *   (as mg_set_scheme) are those of the other entry points.
 * The plan's small device buffers (plan, grid state, potential, twiddles, phase
 * tables, per-workgroup partial sums) live in one file-scope device array of
 * MG_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends; every valid grid
 * fits (a larger plan returns MG_EINVAL).  Calls on one GPU share that array: calls
 * that overlap on one GPU (other threads, other streams) race and must not be made.
 * No device or pinned memory, stream, event or graph is created; the host side uses
 * the C++ heap for the plan's bookkeeping.  Synchronises the stream.  Errors as
 * mg_step (MG_EUNSTABLE leaves psi_dev and the centres unspecified); the message is
 * mg_last_error(NULL).  Results equal those of mg_create + mg_set_state + mg_step on
 * the same input bit for bit. */
#define MG_NOALLOC_SCRATCH_BYTES (1u << 20)
mg_status mg_propagate_noalloc(int D, const int32_t* N, const double* dq, const double* inv_mass, double hbar,
                               mg_precision prec, mg_pot kind, const double* params, int nparams,
                               mg_split split, mg_comp comp, int order, const double* gammas, int nstages,
                               void* psi_dev, double* q_ctr, double* p_ctr, double dt, int64_t nsteps,
                               void* hip_stream);

/* sha256 (hex) of the sources and compile flags the library was built from; the
 * Python binding compares it with the sources beside it and refuses a stale build. */
const char* mg_build_hash(void);

const char* mg_last_error(const void* ctx_or_batch);

#ifdef __cplusplus
}
#endif
#endif /* MGSO_H */
