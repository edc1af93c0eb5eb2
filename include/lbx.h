/*
 * lbx — Lindblad optimal-control hot path for AMD Instinct MI355X (gfx950).
 *
 * C ABI of the library liblbx.so.  Every computation runs in HIP kernels on
 * the current device; this header uses plain C types only.
 *
 * Model (Guenther, Petersson, DuBois, "Quandary", Sec. II and App. A/B):
 *   composite system of Q subsystems with n_q levels, N = prod n_q;
 *   rotating-frame Hamiltonian H(t) = H_sys + sum_q d_q(t) a_q + conj(d_q(t)) a_q^+,
 *   H_sys with detuning, self-Kerr and cross-Kerr terms (diagonal);
 *   collapse operators a_q/sqrt(T1_q) (decay) and a_q^+ a_q/sqrt(T2_q) (dephasing);
 *   controls d_q(t) = sum_s S_s(t) sum_f alpha_q^{s,f} exp(i Omega_q^f t) with
 *   quadratic B-splines S_s on knots of spacing T/(Ns-2), centres (s-1/2)T/(Ns-2).
 *
 * Units: every frequency-like input (detuning, Kerr terms, carriers, control
 * coefficients alpha) is an ordinary frequency in GHz (the value divided by
 * 2*pi); times (T, T1, T2, t) are in ns.  The library multiplies by 2*pi.
 * A decay or dephasing time that is not finite and positive switches its
 * term off.
 *
 * Memory layout shared by every entry point:
 *   - a density matrix rho is complex128, row-major: rho[i][j] at i*N + j,
 *     stored as interleaved (re, im) doubles.  Basis index i has the
 *     subsystem digits of its levels with subsystem 0 most significant.
 *     (The paper's column-stacked vec(rho) is a relabelling of this.)
 *   - a batch of B states of one system is [B][N][N] contiguous;
 *   - a multi-system plan concatenates the batches of its systems in plan
 *     order (batch_per_sys[s] states of system s);
 *   - alpha of one system is [Q][Ns][Nf][2] doubles (Re, Im), flattened;
 *     a multi-system alpha concatenates the systems in plan order; gradients
 *     use the same layout.
 *
 * Ownership: the caller owns every state, alpha, G, grad and workspace
 * buffer.  Pointers documented as DEVICE must be device (or managed) memory
 * of the current device; HOST pointers are read during the call only.
 * A plan owns small immutable device tables (energies, digit tables) and is
 * destroyed with lb_plan_destroy.
 *
 * Streams: `stream` is a hipStream_t (NULL = the default stream).  Kernels
 * are enqueued on it; no entry point synchronises in the middle of its work
 * (the number of stage-solve sweeps of every step is decided on the device).
 * Conditions that only the device sees (a non-finite objective, a step whose
 * stage solve cannot be handled) are raised in a status word at the start
 * of the call's workspace.  With LB_OPT_SYNC on (the default) imr_step,
 * forward_solve, objective, adjoint_backward and adjoint_gradient wait for
 * their work at the end and return that status as their code; with it off
 * they return as soon as the work is enqueued and lb_status() reads the
 * status later.  lindblad_apply and control_table never synchronise.
 * Stage systems whose splitting iteration does not contract (a step with
 * bound theta_j >= 0.5: a large step or control amplitude) are solved with
 * restarted GMRES, as App. A solves every stage system: with LB_OPT_SYNC on
 * a call that meets such a step runs once more with every system streamed,
 * solving those steps with GMRES (a slower path that synchronises at every
 * Krylov step); with it off, lb_status() reports LB_EUNSUPPORTED.
 * Options are copied when a call starts; concurrent calls on one plan (from
 * several threads or streams) need separate workspaces.
 *
 * Errors: every entry point returns LB_OK (0) or a negative code; no C++
 * exception or abort crosses the ABI.  lb_last_error() returns a message for
 * the last failing call of the calling thread.
 */
#ifndef LBX_H
#define LBX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LB_OK 0
#define LB_EINVAL (-1)        /* null pointer, bad size, bad kind, bad option */
#define LB_ENOMEM (-2)        /* workspace too small or device allocation failed */
#define LB_EDEVICE (-3)       /* a HIP call failed; the message has the HIP error */
#define LB_EUNSUPPORTED (-4)  /* inputs outside what the kernels handle */
#define LB_ENONFINITE (-5)    /* NaN or Inf in an objective */

#define LB_J_FROB 0  /* J = 1/2 ||rho_tar - rho||_F^2            (Sec. III, eq. Jmeasure) */
#define LB_J_TR 1    /* J = 1 - Re Tr(rho_tar^+ rho)              (Sec. III, eq. Jmeasure) */
#define LB_J_NM 2    /* J = Re Tr(O^+ rho) = Tr(N_m rho) with the observable O = N_m
                        (diagonal |l - m|) passed in place of rho_tar (Sec. III, eq. Jmeasure) */

/* Workspace queries (lb_workspace_bytes). */
#define LB_OP_IMR_STEP 0
#define LB_OP_FORWARD 1   /* forward_solve, objective */
#define LB_OP_GRADIENT 2  /* adjoint_gradient (the trajectory is kept in the workspace) */
#define LB_OP_BACKWARD 3  /* adjoint_backward (the trajectory is the caller's) */

/* Plan options (lb_plan_set_option). */
#define LB_OPT_PATH 0      /* 0 auto, 1 LDS-resident persistent kernels, 2 streaming sweeps */
#define LB_OPT_SOLVE_TOL 1 /* fixed-point stage-solve bound, default 2^-53 */
#define LB_OPT_PROFILE 2   /* 1: time kernel launches of forward_solve and adjoint_gradient
                              with HIP events on the call's stream; 0 (default): off */
#define LB_OPT_TILE 3      /* 1 (default): block-tiled kernels for large systems of
                              equal-level subsystems; 2: as 1, but lindblad_apply runs
                              the multi-pass kernels where the system has a pass plan;
                              0: generic streaming kernels */
#define LB_OPT_TILE_KI 4   /* block shape of the block-tiled kernels, 10*KR + KC with KR
                              (KC) row (column) digits inside a block; 0 (default): the
                              shape listed first for the system.  100 + KA (KA = 1..Q-1):
                              the two-pass sweeps and apply, pass A over the KA least
                              significant subsystems and pass B over the others */
#define LB_OPT_GRAPH 5     /* > 0: streamed time loops are captured as HIP graphs of this
                              many steps and replayed (one graph launch per chunk);
                              0 (default): kernels are launched directly */
#define LB_OPT_HISTORY 6   /* 0..6, default 5: converged stage increments of earlier steps
                              from which a streamed step extrapolates its first iterate
                              (order HISTORY-1 in the frame of the diagonal Cayley factor);
                              0 starts every stage solve from q */
#define LB_OPT_SYNC 7      /* 1 (default): calls wait for their work and return the device
                              status; 0: calls return once enqueued (see lb_status) */
#define LB_OPT_FUSE_GRAD 9 /* 1: the last sweep of a block-tiled adjoint step also forms the
                              step's gradient integrands (App. B eq. reducedgradient) from the
                              neighbour values it loads, with the stage vector one sweep
                              before convergence (a difference within the stage solve's
                              bound), where the block shape allows it without spilling;
                              0 (default): a separate integrand kernel after the converged
                              step (as fast or faster on the measured systems) */
#define LB_OPT_SWEEPS 8    /* stage-solve sweeps launched per streamed step: 0 (default)
                              8 for steps started from a full history, 12 for the others;
                              2..64: that many for every step.  A step runs only the sweeps
                              its a-posteriori bound asks for; one that needs more than were
                              launched makes an LB_OPT_SYNC call repeat itself once with the
                              a-priori counts of every step read on the host (else lb_status
                              reports LB_EUNSUPPORTED) */

/* Kernel families timed by LB_OPT_PROFILE (lb_profile_read). */
#define LB_KERNEL_LDS_FORWARD 0  /* persistent forward time loop, LDS-resident */
#define LB_KERNEL_LDS_ADJOINT 1  /* persistent adjoint time loop + gradient integrands */
#define LB_KERNEL_SWEEP 2        /* one streamed implicit-midpoint step (all its sweeps) */
#define LB_KERNEL_STREAM_GRAD 3  /* streaming gradient integrands of one step */
#define LB_KERNEL_COUNT 4

#define LB_LIMIT_QMAX 12   /* subsystems per system */
#define LB_LIMIT_NLEV 31   /* levels per subsystem */

/* imr_step_noalloc: its scratch array (bytes per device), the most state
 * entries B*N^2 one call may take, and the most systems its plan may hold. */
#define LB_NOALLOC_SCRATCH_BYTES 67108864
#define LB_NOALLOC_MAX_ENTRIES 2064384
#define LB_NOALLOC_MAX_SYSTEMS 256

/* One composite system (Sec. II).  Host memory; copied by lb_plan_create. */
typedef struct {
  int32_t Q;                /* number of subsystems, 1..LB_LIMIT_QMAX */
  const int32_t *nlev;      /* [Q] levels n_q, 1..LB_LIMIT_NLEV; q = 0 most significant */
  const double *detuning;   /* [Q] (omega_q - omega_q^rot)/2pi [GHz] */
  const double *selfkerr;   /* [Q] xi_q/2pi [GHz]; term -xi_q/2 a^+a^+aa */
  const double *crosskerr;  /* [Q*Q] row-major, entry [p*Q+q] with p<q is xi_pq/2pi [GHz] */
  const double *T1;         /* [Q] decay times [ns] */
  const double *T2;         /* [Q] dephasing times [ns] */
  int32_t Ns;               /* B-spline basis functions per control, >= 3 */
  int32_t Nf;               /* carrier waves per control, >= 1 */
  const double *carrier;    /* [Q*Nf] Omega_q^f/2pi [GHz] */
  double T;                 /* horizon [ns], > 0 */
  int32_t NT;               /* implicit-midpoint steps, >= 1; dt = T/NT */
  const double *jc;         /* [Q*Q] row-major or NULL: entry [p*Q+q] with p>q is the
                               Jaynes-Cummings coupling g_pq/2pi [GHz] (Sec. II) */
  const double *rotfreq;    /* [Q] omega_q^rot/2pi [GHz] or NULL (all equal): the coupling
                               of p > q carries exp(+-i (omega_p^rot - omega_q^rot) t) on
                               a_p^+ a_q and a_p a_q^+ */
} lb_system_desc;

typedef struct lb_plan lb_plan;

/* Validates nsys descriptions and builds the device tables of a plan:
 * per-basis-index energies of H_sys and digit tables.  All systems of one
 * plan must share NT.  Returns LB_EINVAL for invalid descriptions. */
int lb_plan_create(const lb_system_desc *sys, int32_t nsys, lb_plan **out);
void lb_plan_destroy(lb_plan *plan);

/* N, number of real control parameters (2*Q*Ns*Nf) and NT of system `sys`. */
int lb_plan_info(const lb_plan *plan, int32_t sys, int32_t *N, int32_t *nalpha, int32_t *NT);

/* Sets an LB_OPT_* option; options apply to later calls. */
int lb_plan_set_option(lb_plan *plan, int32_t option, double value);

/* Bytes of workspace the operation `op` (LB_OP_*) needs for the batch
 * batch_per_sys[nsys] (HOST).  For LB_OP_IMR_STEP, batch_per_sys may name
 * one system by giving 0 for every other.  ckpt_every is the checkpoint
 * interval of the forward trajectory (LB_OP_GRADIENT, LB_OP_BACKWARD, and
 * LB_OP_FORWARD when forward_solve keeps a trajectory): 0 picks
 * ceil(sqrt(NT)) for streamed systems and keeps every state of the systems
 * small enough for the LDS-resident kernels; 1 keeps every state; c > 1
 * keeps every c-th state of every system (systems that would be
 * LDS-resident are streamed then, since those kernels keep every state).
 * The workspace begins with the call's status word (see lb_status).  The
 * size covers the GMRES fallback of the call (every system streamed). */
int lb_workspace_bytes(const lb_plan *plan, int32_t op, const int32_t *batch_per_sys,
                       int32_t ckpt_every, size_t *bytes);

/* Bytes of the trajectory buffer that forward_solve fills and
 * adjoint_backward reads, for the batch and ckpt_every (as above), in the
 * normal layout or that of the GMRES fallback (the larger of the two). */
int lb_trajectory_bytes(const lb_plan *plan, const int32_t *batch_per_sys, int32_t ckpt_every,
                        size_t *bytes);

/* Waits for `stream` and returns the status that the last call using the
 * workspace `ws` (DEVICE) raised on the device: LB_OK, LB_ENONFINITE (an
 * objective is not finite) or LB_EUNSUPPORTED (a step's stage-solve
 * contraction bound is >= 0.5 in a call that could not fall back to GMRES,
 * a stage solve hit its sweep cap, or a streamed step needed more sweeps
 * than were launched).  With ws NULL: the
 * status of the last imr_step_noalloc call on the current device. */
int lb_status(const lb_plan *plan, const void *ws, void *stream);

/* Launch count and summed duration [ms] of kernel family `kernel` (LB_KERNEL_*)
 * over the calls made while LB_OPT_PROFILE was on; reset != 0 clears them.
 * The stage sweeps of one step are timed together (one event pair around
 * their back-to-back launches), so total_ms / launches is their mean. */
int lb_profile_read(const lb_plan *plan, int32_t kernel, int64_t *launches, double *total_ms,
                    int32_t reset);

/* Work done by kernel family `kernel` over the calls made while
 * LB_OPT_PROFILE was on: state entries times stage-solve sweeps (entries
 * times steps for LB_KERNEL_STREAM_GRAD).  Cleared with lb_profile_read's
 * reset.  Profiling reads the per-state sweep totals of the LDS-resident
 * kernels back after each launch (a synchronisation of the stream). */
int lb_profile_work(const lb_plan *plan, int32_t kernel, int64_t *entry_sweeps);

/* A-priori stage-solve sweep counts per step (HOST counts [nsys][NT][2]:
 * LDS-resident kernels started from w h D q, streaming sweeps started from
 * q) for controls alpha (DEVICE, all systems): the fixed-point stage
 * iteration of the implicit-midpoint solve (App. A) contracts with a factor
 * theta_j that is known before the step, and the count is the number of
 * sweeps after which the contraction bound reaches LB_OPT_SOLVE_TOL.  A count
 * of -1 marks a step with theta_j >= 0.5, solved with GMRES (see Streams).
 * The streaming kernels and the generic LDS-resident kernels run exactly
 * these counts; the specialised LDS-resident kernels start from an
 * extrapolation of the previous stage increments and stop on an
 * a-posteriori bound of the same tolerance.  Synchronises the stream. */
int sweep_counts(const lb_plan *plan, const double *alpha, int32_t *counts, void *stream);

/* Control values d_q(t_{j+1/2}) at every step midpoint of system `sys`
 * (Sec. II eq. rotctrl; App. A: M is evaluated at t_j + dt/2), in rad/ns.
 * alpha: DEVICE [nalpha]; table: DEVICE [NT][Q] complex128. */
int control_table(const lb_plan *plan, int32_t sys, const double *alpha, void *table,
                  void *stream);

/* y = M(t) x, or y = M(t)^+ x when adjoint != 0, for B states of system
 * `sys` (App. A eq. mastereq_vectorized, applied matrix-free).  M^+ is the
 * adjoint for <A, B> = Tr(A^+ B).  alpha: DEVICE [nalpha] of this system;
 * x, y: DEVICE [B][N][N] complex128, must not overlap.  B = 0 is a no-op. */
int lindblad_apply(const lb_plan *plan, int32_t sys, double t, const double *alpha,
                   const void *x, void *y, int32_t B, int32_t adjoint, void *stream);

/* One implicit-midpoint step j (App. A eqs. IMR, linsystem_primal):
 * solves (I - dt/2 M) z = q_in with M = M(t_j + dt/2) and writes
 * q_out = q_in + dt M z.  With adjoint != 0 it takes the adjoint step of
 * App. B eq. linsystem_adjoint: (I - dt/2 M^+) zh = q_in, q_out = q_in + dt M^+ zh.
 * q_in, q_out: DEVICE [B][N][N], distinct.  ws: DEVICE, at least
 * lb_workspace_bytes(LB_OP_IMR_STEP) bytes.  One persistent launch takes the
 * fixed-point sweeps of the stage solve, starting from q_in, as many as the
 * a-posteriori bound after the first sweep asks for (at least two). */
int imr_step(const lb_plan *plan, int32_t sys, int32_t j, const double *alpha, const void *q_in,
             void *q_out, int32_t B, int32_t adjoint, void *ws, size_t ws_bytes, void *stream);

/* imr_step without allocation, for callers that cannot allocate device
 * memory: code under HIP graph capture, allocation-free serving loops.
 * Same step, arguments and results as imr_step with no workspace: its
 * scratch (LB_NOALLOC_SCRATCH_BYTES) is a static device array that every
 * device the library runs on holds until the process ends; it calls no
 * hipMalloc or hipFree.  B*N^2 must not exceed LB_NOALLOC_MAX_ENTRIES and the
 * plan must hold at most LB_NOALLOC_MAX_SYSTEMS systems (else LB_EINVAL).
 * Every call on a device shares that device's scratch (which keeps the last
 * call's contents): calls that overlap on one device race.  With LB_OPT_SYNC
 * off the call returns once enqueued and lb_status(plan, NULL, stream) reads
 * its status. */
int imr_step_noalloc(const lb_plan *plan, int32_t sys, int32_t j, const double *alpha, const void *q_in,
                     void *q_out, int32_t B, int32_t adjoint, void *stream);

/* Integrates every state of every system from t = 0 to T (App. A).
 * alpha: DEVICE, all systems concatenated; rho0, rhoT: DEVICE batched states;
 * batch_per_sys: HOST [nsys].  traj: DEVICE buffer of lb_trajectory_bytes
 * bytes that receives the forward states adjoint_backward needs (checkpoints
 * every ckpt_every steps, see lb_workspace_bytes), or NULL (ckpt_every is
 * then ignored).  ws: DEVICE, lb_workspace_bytes(LB_OP_FORWARD, ckpt_every). */
int forward_solve(const lb_plan *plan, const double *alpha, const void *rho0, void *rhoT,
                  const int32_t *batch_per_sys, void *traj, int32_t ckpt_every, void *ws,
                  size_t ws_bytes, void *stream);

/* G_s = (1/M_s) sum_i beta_i J(rho_tar_i, rho_i(T)) + gamma2/2 ||alpha_s||^2 for
 * every system s (Sec. III eq. optimproblem with gamma1 = 0: the running
 * penalty needs the whole trajectory, adjoint_gradient computes it),
 * M_s = batch_per_sys[s].
 * rhoT, rhotar: DEVICE batched states; beta: DEVICE [total states];
 * alpha: DEVICE; G: DEVICE [nsys]; J: DEVICE [total states] or NULL, receives
 * each J_i (unweighted).  ws: DEVICE, lb_workspace_bytes(LB_OP_FORWARD).
 * The status (LB_OPT_SYNC, lb_status) is LB_ENONFINITE when a G is not finite. */
int objective(const lb_plan *plan, int32_t kind, const void *rhoT, const void *rhotar,
              const double *beta, const int32_t *batch_per_sys, double gamma2,
              const double *alpha, double *G, double *J, void *ws, size_t ws_bytes,
              void *stream);

/* Adjoint pass and exact discrete gradient (App. B eqs. linsystem_adjoint,
 * reducedgradient) from a trajectory that forward_solve kept with the same
 * ckpt_every: terminal condition (beta_i/M) dJ/d(conj q) at the rho(T) of the
 * trajectory, adjoint implicit-midpoint steps backwards with the forward
 * states recomputed between checkpoints, and
 *   grad = sum_s gscale[s] (dG_s/dalpha_s)   (gscale NULL: all ones),
 * which is the backward pass of G for an incoming gradient gscale (the
 * adjoint is linear in its terminal condition).  gscale: DEVICE [nsys] or
 * NULL; grad: DEVICE like alpha.  ws: DEVICE, lb_workspace_bytes(LB_OP_BACKWARD). */
int adjoint_backward(const lb_plan *plan, int32_t kind, const double *alpha, const void *traj,
                     int32_t ckpt_every, const void *rhotar, const double *beta,
                     const int32_t *batch_per_sys, double gamma2, const double *gscale,
                     double *grad, void *ws, size_t ws_bytes, void *stream);

/* Objective and its exact discrete gradient (App. B eqs. linsystem_adjoint,
 * reducedgradient): forward solve with checkpoints, terminal condition
 * (beta_i/M) dJ/d(conj q), adjoint implicit-midpoint sweep backwards with
 * recomputation between checkpoints, and the gradient reduction
 * dG/dalpha = sum_j dt Re <zh^j, dM/dalpha z^j> + gamma2 alpha.
 * gamma1 != 0 adds the running penalty of Sec. III eq. optimproblem,
 *   gamma1 (1/M_s) sum_i dt sum_{j=0}^{NT-1} beta(t_j) J(rho_tar_i, q_i^j),
 *   beta(t) = exp(-((t - T)/a)^2) / a,  a = penalty_a > 0 [ns],
 * the time integral taken by the left rectangle rule on the step grid and
 * averaged over the initial states without the weights beta_i; the adjoint
 * then carries its source term gamma1 dt beta(t_j) (1/M) dJ/d(conj q^j)
 * (App. B).  With it, LDS-resident systems run on the generic LDS kernels.
 * G: DEVICE [nsys]; grad: DEVICE like alpha; rhoT: DEVICE batched states or
 * NULL.  ws: DEVICE, lb_workspace_bytes(LB_OP_GRADIENT, ckpt_every) bytes.
 * Errors: LB_EINVAL for a non-finite gamma1 or gamma2, or (gamma1 != 0) a
 * penalty_a that is not positive and finite.  The status (LB_OPT_SYNC) is
 * LB_ENONFINITE when a G is not finite. */
int adjoint_gradient(const lb_plan *plan, int32_t kind, const double *alpha, const void *rho0,
                     const void *rhotar, const double *beta, const int32_t *batch_per_sys,
                     double gamma2, double gamma1, double penalty_a, int32_t ckpt_every, double *G,
                     double *grad, void *rhoT, void *ws, size_t ws_bytes, void *stream);

/* Autotuner for the streamed systems of batch_per_sys (HOST): times a few
 * implicit-midpoint steps of the generic step kernel and of every
 * instantiated block shape of the block-tiled one on the workspace (DEVICE,
 * lb_workspace_bytes(LB_OP_FORWARD) bytes; its contents are overwritten), and
 * sets LB_OPT_TILE and LB_OPT_TILE_KI of the plan to the fastest.  result:
 * HOST [3], the values of LB_OPT_TILE, LB_OPT_TILE_KI and LB_OPT_GRAPH.
 * alpha: DEVICE.  Synchronises the stream.  A plan without streamed systems
 * in this batch is left unchanged. */
int lb_autotune(lb_plan *plan, const double *alpha, const int32_t *batch_per_sys, void *ws,
                size_t ws_bytes, void *stream, int32_t *result);

/* Message for the last non-zero return on the calling thread ("" if none). */
const char *lb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LBX_H */
