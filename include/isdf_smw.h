/*
 * isdf_smw.h -- C ABI of the MI355X (gfx950) ISDF-SMW dielectric-inverse library.
 *
 * The library computes the inverse of the symmetrised dielectric matrix
 *     eps~ = I - V^{1/2} chi0 V^{1/2}
 * in a plane-wave basis, with chi0 = f M_vc W M_vc^H built from the
 * valence-conduction pair products M_vc(r; i, j) = conj(psi_i(r)) psi_j(r)
 * (paper, Sec. 2, eq. matrices and eq. Omega) and W = diag(w_ij),
 * w_ij = Delta_ij / (Delta_ij^2 + omega^2), Delta_ij = eps_i - eps_j < 0
 * (omega = 0: the static Omega^{-1}; omega > 0: the imaginary-frequency
 * weight that follows from the two pole terms of eq. Hedin_fourier).
 *
 * The method (paper, Sec. "ISDF" and Sec. "SMW formula combined with ISDF",
 * eq. epsilon_with_SMW, and the matrix K of Sec. "Cubic scaling algorithm"):
 *   1. ISDF fit: M_vc ~ Theta C, C(mu; i, j) = conj(psi_i(r_mu)) psi_j(r_mu)
 *      (eq. ISDF, eq. MatrixExpressionISDF), Theta the least-squares fit
 *      Theta (C C^H) = M_vc C^H, whose two factors are Hadamard products of
 *      orbital Gram blocks (the identity of eq. Hadamard);
 *   2. core M = f C W C^H (eq. COmegaCstar times f), N_mu x N_mu;
 *   3. Coulomb-weighted U = V^{1/2} (F Theta) on the plane-wave list, with F
 *      the unitary grid DFT, and U^H U = Theta^H V Theta;
 *   4. SMW: eps~^{-1} = I + U (M^{-1} - U^H U)^{-1} U^H.
 *
 * Conventions shared by every entry point
 *   - All functions return isdf_status.  No exception crosses the ABI.
 *   - "device" pointers are HIP device memory on the handle's device; "host"
 *     pointers are ordinary host memory, read before the call returns.
 *   - The caller owns every input, output and workspace buffer.  The library
 *     allocates no device memory after isdf_create and frees no caller memory.
 *   - Work is enqueued on the handle's stream.  Entry points that produce a
 *     result synchronise that stream once at the end to read the device status
 *     word; outputs are unspecified when the return value is not ISDF_OK.
 *   - Argument errors are found on the host before anything is enqueued
 *     (ISDF_E_ARG, message in isdf_last_error).
 *   - Complex numbers are interleaved (re, im) pairs of double.
 *   - Orbitals: psi is Nr x N column-major, i.e. psi[n * Nr + k] = psi_n(r_k),
 *     a (N, Nr) C-contiguous array; states 0..nv-1 occupied, nv..nv+nc-1
 *     empty; grid index k = i0 + n0 (i1 + n1 i2).  Columns should be
 *     orthonormal in the plain grid inner product (quadrature weights are
 *     dropped, as in the paper; v_scale restores physical units).
 *   - Plane waves: miller is ng x 3 int32 (m_x, m_y, m_z), each component in
 *     [-n_d/2, n_d/2), distinct; G = 2 pi B m with B the reciprocal basis of
 *     the cell rows.  V(G) = v_scale 4 pi / |G|^2 and V(0) = 0.
 *   - Calls on one handle must not overlap in time; different handles may be
 *     used from different host threads.
 */
#ifndef ISDF_SMW_H
#define ISDF_SMW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct isdf_handle_s* isdf_handle;
typedef struct isdf_plan_s* isdf_plan;
typedef struct isdf_graph_s* isdf_graph;

typedef enum {
  ISDF_OK = 0,
  ISDF_E_ARG = -1,         /* invalid argument (host check, nothing enqueued) */
  ISDF_E_NOT_PD = -2,      /* a Hermitian matrix that must be positive definite was not */
  ISDF_E_DEVICE = -3,      /* HIP runtime error */
  ISDF_E_WORKSPACE = -4,   /* workspace NULL, too small or misaligned (256 B) */
  ISDF_E_UNSUPPORTED = -5  /* valid request the library does not implement */
} isdf_status;

typedef enum {
  ISDF_FP64 = 0,    /* every contraction in FP64 on MFMA */
  ISDF_FP32 = 1,    /* large contractions in FP32 on MFMA, FP32 accumulation; N_mu x N_mu core in FP64 */
  ISDF_BF16X3 = 2   /* the pair-Gram contraction of step 1 and the core M of step 2 as three BF16 products
                       (hi*hi + hi*lo + lo*hi, x = hi + lo split by round to nearest) on bf16 MFMA with
                       FP32 accumulation (the core's per-state sums added in FP64); the other large
                       contractions as ISDF_FP32; N_mu x N_mu algebra in FP64 */
} isdf_precision;

typedef struct {
  int32_t n[3];          /* FFT grid; Nr = n[0] n[1] n[2]; each in [2, 1024]; the calls that
                            take a plane-wave list need each <= 64 (else ISDF_E_UNSUPPORTED) */
  double cell[9];        /* lattice vectors as rows, Bohr */
  int32_t nv, nc;        /* occupied / empty state counts, both >= 1 */
  int32_t is_complex;    /* 0: psi is real float64; 1: psi is complex128 */
  double pair_factor;    /* f in chi0 = f M W M^H; the paper's value is 2 */
  double v_scale;        /* Coulomb prefactor; Nr / cell volume for unit-norm grid orbitals */
  int32_t prec;          /* isdf_precision */
  int32_t refine_steps;  /* FP64 Newton refinement steps T <- T + T (I - H T) on the core inverse, 0..8 */
  int32_t coulomb_sum;   /* plane waves the Coulomb Gram sums over (the P^H V P of Algorithm 3,
                            step 2, inside eq. epsilon_with_SMW):
                            0: the ng-vector list (the truncated basis, default);
                            1: every grid vector, the paper's P^H V P over the whole FFT grid.
                            The output is the ng x ng block over the list in both cases; with 1
                            the workspace grows with Nr (isdf_workspace_bytes accounts for it).
                            Read by the calls that take a plane-wave list (isdf_eps_inv,
                            isdf_coulomb_u, isdf_plan_create); isdf_smw_apply sums over the
                            rows of the U it is given. */
  int32_t core_method;   /* how the core M = f C Omega^{-1} C^H is formed:
                            0: the direct pair sum over every (i, j) (eq. COmegaCstar, default);
                            1: the contour integral of Algorithm 2 (static only: isdf_eps_inv
                               with n_omega = 0, isdf_core_m with omega = 0; plans and the
                               adjoint return ISDF_E_UNSUPPORTED).  Cost N_lambda (Nv + Nc)
                               N_mu^2 instead of Nv Nc N_mu^2 / 2 */
  double core_tol;       /* core_method 1: quadrature tolerance; the node count N_lambda is the
                            smallest with exp(-pi^2 N / (2 log(Q/q) + 6)) <= core_tol
                            (eq. rel_err_Cauchy; q gap, Q span of the empty band; at most 256).
                            0 selects 1e-13; must be < 1e-2 */
} isdf_problem;

typedef struct {
  double stage_ms[8];        /* filled when want_timing != 0: HIP-event intervals on the caller's stream.
                                isdf_eps_inv: [0] point gather, first core M, operand conversion, [1] the pair
                                product Z (exactly one kernel launch), [2] DFT to X = V^{1/2} F Z,
                                [3] X^H X, [4] core solve (waits for K = S M^{-1} S from the
                                library's second stream, H = X^H X - K, H^{-1}, refinement),
                                [5] W = X H^{-1}, [6] output, [7] unused.
                                S, the DFT tables, M^{-1} and K (and the later frequencies' cores
                                M) run concurrently on a library-owned stream.
                                isdf_smw_apply: [0] input conversion and M^{-1}, [1] zero,
                                [2] U^H U, [3] core solve, [4] U T, [5] output. */
  double refine_residual[9]; /* ||I - H T_k||_F / sqrt(N_mu) for k = 0..refine_steps (last frequency),
                                T_k the k-th Newton-refined H^{-1}; H = X^H X - S M^{-1} S
                                (isdf_eps_inv) or U^H U - M^{-1} (isdf_smw_apply) */
  double min_pivot;          /* smallest diagonal entry of H (last frequency) */
  int32_t want_timing;       /* input: 1 to record per-stage HIP events (adds host syncs) */
  int32_t n_refine_reported; /* number of valid refine_residual entries */
  double cond_est;           /* ||H||_F ||H^{-1}||_F of the last frequency, an upper bound on the
                                2-norm condition number of the core H (isdf_eps_inv, isdf_smw_apply,
                                plans); the core inverse loses about log10(cond_est) digits */
} isdf_report;

/* Create a handle bound to HIP device `device` and stream `hip_stream`
 * (a hipStream_t; NULL = default stream).  Allocates only a small pinned
 * host staging buffer and a few events.  Errors: ISDF_E_ARG (h NULL or bad
 * device), ISDF_E_DEVICE. */
isdf_status isdf_create(isdf_handle* h, int device, void* hip_stream);

/* Destroy a handle; waits for its stream.  NULL is accepted. */
isdf_status isdf_destroy(isdf_handle h);

/* Rebind the handle to another stream on the same device. */
isdf_status isdf_set_stream(isdf_handle h, void* hip_stream);

/* Device workspace bytes needed by isdf_eps_inv and the stage calls for this
 * problem, n_mu interpolation points, ng plane waves and n_omega frequencies
 * (0 = static).  Host only; does not need a handle or a GPU. */
isdf_status isdf_workspace_bytes(const isdf_problem* prob, int32_t n_mu, int32_t ng,
                                 int32_t n_omega, size_t* bytes);

/* The first ng Miller vectors of the grid, ordered by (|m|^2, m_x, m_y, m_z)
 * ascending, each component in [-n_d/2, n_d/2).  Host only.  miller_out: host,
 * ng x 3 int32, caller-allocated. */
isdf_status isdf_gvectors(const isdf_problem* prob, int32_t ng, int32_t* miller_out);

/* eps~^{-1} for each requested frequency (paper: eq. epsilon_with_SMW with
 * the ISDF pair products; steps 1-4 above, all on the GPU).
 *   psi       device, Nr x N (see conventions), float64 or complex128 per is_complex
 *   energies  host, N doubles (Hartree); max over occupied < min over empty
 *   mu_idx    host, n_mu distinct grid indices in [0, Nr); 1 <= n_mu <= nv*nc
 *   miller    host, ng x 3 int32, distinct, in range; 1 <= ng <= Nr
 *   omega     host, n_omega imaginary frequencies (Hartree, >= 0); NULL with
 *             n_omega = 0 means one static (omega = 0) result
 *   workspace device, >= isdf_workspace_bytes(...), 256-byte aligned
 *   eps_inv   device out, max(n_omega, 1) x ng x ng complex128, C order:
 *             eps_inv[w][g][g'] = eps~^{-1}(G_g, G_g') at omega_w.  Exactly
 *             Hermitian (lower triangle computed, upper mirrored).
 *   rep       host out, optional (NULL)
 * Errors: ISDF_E_ARG, ISDF_E_WORKSPACE, ISDF_E_NOT_PD (C C^H or -M not
 * positive definite, e.g. points that make C rank deficient), ISDF_E_DEVICE. */
isdf_status isdf_eps_inv(isdf_handle h, const isdf_problem* prob, const void* psi,
                         const double* energies, const int32_t* mu_idx, int32_t n_mu,
                         const int32_t* miller, int32_t ng, const double* omega,
                         int32_t n_omega, void* workspace, size_t ws_bytes, void* eps_inv,
                         isdf_report* rep);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): isdf_eps_inv with no
 * workspace argument.  The workspace is a library-owned device array of
 * ISDF_SCRATCH_MAX_BYTES per GPU, set up by isdf_create and held until the
 * process ends; this call allocates nothing (device or pinned host memory).
 * Every call on one GPU uses that GPU's one array: calls that overlap on a GPU
 * (on different streams or handles) race and give undefined results.  The
 * array keeps the last call's contents; the call clears what must start at zero.
 * Arguments as for isdf_eps_inv.  Errors: those of isdf_eps_inv, and
 * ISDF_E_WORKSPACE (with a message) when the problem needs more than
 * ISDF_SCRATCH_MAX_BYTES (isdf_workspace_bytes tells beforehand) or its host
 * arrays do not fit the handle's pinned staging buffer (1 MiB); nothing is
 * enqueued then. */
#define ISDF_SCRATCH_MAX_BYTES ((size_t)64 << 20)
isdf_status isdf_eps_inv_noalloc(isdf_handle h, const isdf_problem* prob, const void* psi,
                                 const double* energies, const int32_t* mu_idx, int32_t n_mu,
                                 const int32_t* miller, int32_t ng, const double* omega,
                                 int32_t n_omega, void* eps_inv, isdf_report* rep);

/* Step 1 alone: Theta in real space (eq. ISDF, least-squares fit).
 *   theta  device out, N_mu x Nr complex128 C order: theta[mu][k] = Theta(r_k, mu).
 * Other arguments as for isdf_eps_inv. */
isdf_status isdf_fit_theta(isdf_handle h, const isdf_problem* prob, const void* psi,
                           const int32_t* mu_idx, int32_t n_mu, void* workspace,
                           size_t ws_bytes, void* theta);

/* Step 2 alone: the core M = f C W C^H (eq. COmegaCstar times f) at one frequency.
 *   m_out  device out, N_mu x N_mu complex128 C order (Hermitian, negative definite). */
isdf_status isdf_core_m(isdf_handle h, const isdf_problem* prob, const void* psi,
                        const double* energies, const int32_t* mu_idx, int32_t n_mu,
                        double omega, void* workspace, size_t ws_bytes, void* m_out);

/* Steps 1 and 3: U = V^{1/2} (F Theta) restricted to the plane-wave list.
 *   u_out  device out, ng x N_mu complex128 C order: u[g][mu]. */
isdf_status isdf_coulomb_u(isdf_handle h, const isdf_problem* prob, const void* psi,
                           const int32_t* mu_idx, int32_t n_mu, const int32_t* miller,
                           int32_t ng, void* workspace, size_t ws_bytes, void* u_out);

/* Step 4 alone: eps~^{-1} = I + U (M^{-1} - U^H U)^{-1} U^H from given U and M
 * (eq. epsilon_with_SMW, symmetrised).
 *   u      device, ng x N_mu complex128 C order
 *   m      device, N_mu x N_mu complex128 C order, Hermitian negative definite
 *   eps_inv device out, ng x ng complex128. */
isdf_status isdf_smw_apply(isdf_handle h, const isdf_problem* prob, const void* u,
                           const void* m, int32_t n_mu, int32_t ng, void* workspace,
                           size_t ws_bytes, void* eps_inv, isdf_report* rep);

/* ---- Plans: the same path as isdf_eps_inv, set up once, enqueued many times ----
 *
 * A plan holds everything about a problem that does not change between calls:
 * the validated problem, the interpolation points, the plane-wave list, the
 * pruned-DFT index tables and the workspace layout.  isdf_plan_create checks
 * these inputs on the host (same rules as isdf_eps_inv), builds the tables and
 * copies them into a small device buffer the caller provides (its size from
 * isdf_plan_table_bytes); the plan also keeps its device status block there.
 *
 * isdf_plan_eps_inv then only enqueues work on the handle's stream: no host
 * synchronisation, no host-to-device copy, so a loop of calls keeps the GPU
 * busy back to back.  Errors found on the device (no gap in the energies, a
 * matrix that is not positive definite) accumulate in the plan's status and
 * are returned by the next isdf_plan_sync, which waits for the stream, then
 * clears the status.  Calls of one plan must not overlap on different streams,
 * and each call's workspace must not be in use by another call still in flight
 * (calls on one stream are ordered, so one workspace can serve a whole loop). */

/* Device bytes of a plan's tables for these arguments (host only, no handle or
 * GPU needed; arguments as for isdf_plan_create).  Errors as isdf_plan_create's
 * host checks: ISDF_E_ARG, ISDF_E_UNSUPPORTED. */
isdf_status isdf_plan_table_bytes(const isdf_problem* prob, const int32_t* mu_idx, int32_t n_mu,
                                  const int32_t* miller, int32_t ng, int32_t n_omega, size_t* bytes);

/* Create a plan for `prob` with n_mu points mu_idx, ng plane waves miller and
 * n_omega frequencies per call (0 = static); arguments as for isdf_eps_inv
 * (host arrays, copied).
 *   tables       device, caller-owned, >= isdf_plan_table_bytes(...), 256-byte aligned;
 *                written here (a copy on the handle's stream, then a stream
 *                synchronisation) and used by every call of the plan, so it must
 *                stay allocated and untouched until isdf_plan_destroy
 *   table_bytes  its size
 * Errors: ISDF_E_ARG, ISDF_E_UNSUPPORTED, ISDF_E_WORKSPACE (tables NULL, too
 * small or misaligned), ISDF_E_DEVICE. */
isdf_status isdf_plan_create(isdf_handle h, const isdf_problem* prob, const int32_t* mu_idx,
                             int32_t n_mu, const int32_t* miller, int32_t ng, int32_t n_omega,
                             void* tables, size_t table_bytes, isdf_plan* plan);

/* Destroy a plan (waits for the streams of its calls).  NULL is accepted.  The
 * table buffer stays the caller's. */
isdf_status isdf_plan_destroy(isdf_plan plan);

/* Device workspace bytes one isdf_plan_eps_inv call needs. */
isdf_status isdf_plan_workspace_bytes(isdf_plan plan, size_t* bytes);

/* Enqueue eps~^{-1} for the plan's problem (paper: eq. epsilon_with_SMW with the
 * ISDF pair products, the same kernels as isdf_eps_inv).
 *   psi       device, as for isdf_eps_inv
 *   energies  DEVICE, N doubles (Hartree); the gap is checked on the device
 *   omega     host, the plan's n_omega frequencies (read during the call); NULL if 0
 *   workspace device, >= isdf_plan_workspace_bytes, 256-byte aligned
 *   eps_inv   device out, max(n_omega, 1) x ng x ng complex128, as for isdf_eps_inv
 * Returns host-side argument errors (ISDF_E_ARG, ISDF_E_WORKSPACE) at once;
 * device-side ones at the next isdf_plan_sync. */
isdf_status isdf_plan_eps_inv(isdf_plan plan, const void* psi, const double* energies,
                              const double* omega, void* workspace, size_t ws_bytes, void* eps_inv);

/* Several systems (possibly of different sizes) in one call: plans[i] with its
 * own arguments psi[i], energies[i], omega[i] (omega may be NULL when no plan
 * has frequencies), workspace[i] / ws_bytes[i], eps_inv[i], each as for
 * isdf_plan_eps_inv.  The work of plans whose handles are bound to other
 * streams is forked off plans[0]'s stream and joined back into it, so the
 * systems run concurrently; plans sharing a handle run one after another.  All
 * plans must be on one device.  Only enqueues; each plan reports its own
 * device errors at its next isdf_plan_sync.
 * Stream capture: when plans[0]'s stream is capturing, every plan must be bound
 * to that same stream (the systems then run one after another in the graph);
 * otherwise ISDF_E_UNSUPPORTED and nothing is enqueued.  For concurrent systems
 * in one graph use isdf_multi_graph_create. */
isdf_status isdf_plan_eps_inv_multi(int32_t count, const isdf_plan* plans, const void* const* psi,
                                    const double* const* energies, const double* const* omega,
                                    void* const* workspace, const size_t* ws_bytes, void* const* eps_inv);

/* Several systems as one instantiated HIP graph whose systems run concurrently.
 * Arguments as for isdf_plan_eps_inv_multi; they are baked into the graph, so
 * every buffer must stay allocated while the graph exists, and each system
 * needs its own workspace and output (ISDF_E_ARG otherwise).  Each plan's call
 * is captured on its own handle's stream (which must be a created stream, not
 * the null stream); the captured kernels and their dependencies are copied into
 * one parent graph, with no dependencies between the systems (a capture holding
 * other node kinds is added as a child graph instead).  Capturing enqueues
 * nothing; stage timing is not recorded inside the graph.  Errors: ISDF_E_ARG,
 * ISDF_E_WORKSPACE, ISDF_E_DEVICE (a capture, copy or instantiation error). */
isdf_status isdf_multi_graph_create(int32_t count, const isdf_plan* plans, const void* const* psi,
                                    const double* const* energies, const double* const* omega,
                                    void* const* workspace, const size_t* ws_bytes,
                                    void* const* eps_inv, isdf_graph* graph);

/* Launch the graph on `hip_stream` (a hipStream_t, NULL = null stream).  The
 * plans' next isdf_plan_sync waits for that stream and returns the device errors
 * of the launch.  Launches of one graph must not overlap. */
isdf_status isdf_graph_launch(isdf_graph graph, void* hip_stream);

/* Destroy the graph (NULL is accepted); the plans and buffers stay the caller's. */
isdf_status isdf_graph_destroy(isdf_graph graph);

/* Launch-shape knobs of a plan (a project-written autotuner chooses them):
 *   dft_zb          z-planes per workgroup of the DFT, 1..64 (default 8); the fused
 *                   x/y/z pass raises it to at least ceil(n[2] / 8)
 *   core_split_pct  split of the core M over the occupied index, percent of the
 *                   built-in choice, 25..200 (default 100)
 *   gram_split      cap on the split-K factor of X^H X, 1..16 (default 8)
 *   wg_per_cu       workgroups per CU of the persistent single-precision kernels, 1..4
 *                   (default 1)
 *   core_stream     where the first frequency's core M runs: 0 on the caller's stream
 *                   before the pair kernel (default), 1 on the library's second stream
 *                   after it, beside the DFT and X^H X, 2 on the second stream right
 *                   after the pair kernel's operand pass, beside the pair kernel
 *   side_prio       1 (default): the Gauss-Jordan sweep steps on the library's second
 *                   stream raise their waves' issue priority over the kernels they share
 *                   the CUs with; 0: they run at normal priority
 *   dft_pipe        single precision: 1 (default) runs the DFT to X as a warp-specialised
 *                   pass (matrix-core waves transform a slab while other waves sum the
 *                   previous one) where the grid shape allows, 0 the single-role pass
 *   best_ms         output of isdf_plan_autotune: time of one call with the chosen knobs */
typedef struct {
  int32_t dft_zb;
  int32_t core_split_pct;
  int32_t gram_split;
  int32_t wg_per_cu;
  int32_t core_stream;
  int32_t side_prio;
  int32_t dft_pipe;
  double best_ms;
} isdf_tune;

/* Set or read a plan's knobs (best_ms is ignored / returned as 0).  Knobs change
 * launch shapes and split orders only; results change at most by rounding. */
isdf_status isdf_plan_set_tune(isdf_plan plan, const isdf_tune* tune);
isdf_status isdf_plan_get_tune(isdf_plan plan, isdf_tune* tune);

/* Autotune a plan on real arguments (as for isdf_plan_eps_inv): times `reps`
 * enqueued calls per candidate with HIP events on the handle's stream, going
 * over the knobs one at a time (coordinate descent, each knob over a fixed
 * candidate list) and keeping the fastest; a candidate replaces the current
 * choice only when it is at least 0.5% faster, so timing noise does not move
 * the knobs.  Leaves the plan set to the choice and returns it in `out`
 * (optional).  Synchronises the stream. */
isdf_status isdf_plan_autotune(isdf_plan plan, const void* psi, const double* energies, const double* omega,
                               void* workspace, size_t ws_bytes, void* eps_inv, int32_t reps, isdf_tune* out);

/* Wait for the stream of the plan's last call (or graph launch) and return the
 * first error any call enqueued since the previous sync found on the device: ISDF_E_ARG (energies without a
 * gap or not finite), ISDF_E_NOT_PD; then clear it.  rep (optional) receives
 * the last call's min_pivot and refinement residuals, and, with stage timing
 * on, stage_ms = the mean of each stage's HIP-event interval over the calls
 * since the previous sync (zeros otherwise). */
isdf_status isdf_plan_sync(isdf_plan plan, isdf_report* rep);

/* Stage timing of a plan's calls: on = 1 makes each call record HIP events at
 * its stage boundaries on the handle's stream (the stages of isdf_report;
 * at most 256 calls between two syncs are timed), on = 0 stops it.  For
 * measurement; not for calls inside a stream capture.  Errors: ISDF_E_ARG. */
isdf_status isdf_plan_time_stages(isdf_plan plan, int32_t on);

/* Host-only check of every host-side argument of isdf_eps_inv (problem, energies,
 * points, plane waves, frequencies); no GPU or handle needed.  Returns the
 * status isdf_eps_inv would return for these arguments before enqueueing
 * anything; msg (optional, host, msg_len bytes) receives the error text. */
isdf_status isdf_check_inputs(const isdf_problem* prob, const double* energies,
                              const int32_t* mu_idx, int32_t n_mu, const int32_t* miller,
                              int32_t ng, const double* omega, int32_t n_omega, char* msg,
                              size_t msg_len);

/* Host only: the contour rule of core_method 1 for these energies (Algorithm 2).
 * The nodes lie on the upper half of the elliptic-map contour around the empty
 * band, q = eps[nv] - eps[nv-1], Q = eps[nv+nc-1] - eps[nv-1] (the energies must
 * be sorted at the band edges: eps[nv-1] the largest occupied, eps[nv] the
 * smallest empty).  out (host, 4 * 256 doubles) receives n lambdas then n
 * quadrature weights, each as (re, im), ordered from the low-energy end; n_out the
 * node count.  Errors: ISDF_E_ARG. */
isdf_status isdf_contour_nodes(const double* energies, int32_t nv, int32_t nc, double tol, double* out,
                               int32_t* n_out);

/* ---- Adjoint of one build ---------------------------------------------------
 * Gradients of the scalar loss L = Re tr(W eps~^{-1}) for a Hermitian weight W,
 * eps~^{-1} the NG x NG result of isdf_eps_inv at one imaginary frequency omega
 * (0 = static).  The derivative is taken of the whole chain: the ISDF fit
 * (eq. MatrixExpressionISDF), the core M = f C Omega^{-1} C^H (eq. COmegaCstar),
 * the Coulomb Gram through the DFT and the SMW update (eq. epsilon_with_SMW).
 * The Nr x N_mu pair products are recomputed from psi, not stored: nothing of
 * an earlier forward call is needed.  They exist for one chunk of interpolation
 * points at a time (at most 512 MiB each), so the workspace grows with N_mu Nr only
 * through that chunk.
 *   prob        prec ISDF_FP64 (every step in FP64) or ISDF_FP32 (the contractions
 *               over the grid, those that form the pair products and those that
 *               contract their cotangents with psi, in FP32 on MFMA with FP64
 *               storage; everything else in FP64); ISDF_BF16X3 is
 *               ISDF_E_UNSUPPORTED; coulomb_sum 0 or 1
 *   psi, energies, mu_idx, n_mu, miller, ng   as for isdf_eps_inv
 *   omega       host, one frequency >= 0 (Hartree)
 *   w           device, ng x ng complex128 row-major, Hermitian (read only)
 *   workspace   device, >= isdf_grad_workspace_bytes, 256-byte aligned
 *   grad_energies  device out, N doubles: dL/d eps_n
 *   grad_psi_mu    device out, N x n_mu complex128 row-major: [n][mu] =
 *                  dL/dRe psi_n(r_mu) + i dL/dIm psi_n(r_mu), the total derivative
 *                  with respect to the orbital value at each interpolation point
 *                  (through C, S, M and the grid rows of the pair products)
 *   loss        host out, optional: L
 * Synchronises the handle's stream.  Errors: ISDF_E_ARG, ISDF_E_WORKSPACE,
 * ISDF_E_UNSUPPORTED, ISDF_E_NOT_PD (S, -M or U^H U - M^{-1} not positive
 * definite), ISDF_E_DEVICE; outputs unspecified on error. */
isdf_status isdf_grad_workspace_bytes(const isdf_problem* prob, int32_t n_mu, int32_t ng,
                                      size_t* bytes);
isdf_status isdf_eps_inv_grad(isdf_handle h, const isdf_problem* prob, const void* psi,
                              const double* energies, const int32_t* mu_idx, int32_t n_mu,
                              const int32_t* miller, int32_t ng, double omega, const void* w,
                              void* workspace, size_t ws_bytes, double* grad_energies,
                              void* grad_psi_mu, double* loss);

/* Static COHSEX self-energy diagonals (paper: Algorithm 3, steps 2 and 4-7; the
 * self-energy terms of eq. selfenergySum in the matrix form of eq. classical56,
 * reduced by eq. Hadamard).  For every band n (N = nv + nc):
 *   Sigma_SEX_X(n) = - sum_{i in v}   m_in^H (W - V) m_in,
 *   Sigma_X(n)     = - sum_{i in v}   m_in^H  V      m_in,
 *   Sigma_COH(n)   = 1/2 sum_{i in all} m_in^H (W - V) m_in,
 * with the pair functions m_in = conj(psi_i) psi_n replaced by their ISDF fits on two
 * more point sets: mu_vn for the occupied x all pairs (P_vn) and mu_nn for the all x
 * all pairs (P_nn), each fitted by least squares like the valence-conduction set.
 * W - V = V^{1/2} (eps~^{-1} - I) V^{1/2} on the plane-wave list, with eps~^{-1} the
 * static result of isdf_eps_inv for mu_idx (written to eps_inv on the way); V is the
 * same list's Coulomb operator, for the bare exchange too.  The screened part enters
 * in Algorithm 3's low-rank form (P_s^H V P_vc) K (P_s^H V P_vc)^H; no NG x NG matrix
 * is read.  Arguments as for isdf_eps_inv (static: no frequencies), and
 *   mu_vn, mu_nn  host, distinct grid indices; 1 <= n_mu_vn <= nv N and
 *                 1 <= n_mu_nn <= N^2 (and <= Nr)
 *   workspace     device, >= isdf_sigma_workspace_bytes(...), 256-byte aligned
 *   eps_inv       device out, ng x ng complex128 (as isdf_eps_inv)
 *   sigma         device out, 3 x N doubles (Hartree): [0] Sigma_SEX_X, [1] Sigma_X,
 *                 [2] Sigma_COH (each diagonal is real: Hermitian forms)
 * ISDF_FP64 runs every step in FP64; ISDF_FP32 and ISDF_BF16X3 run the self-energy
 * sets' contractions over the grid and the plane waves in FP32 (complex64 storage)
 * and their N_mu-sized algebra in FP64.  Synchronises the handle's stream.
 * Errors: those of isdf_eps_inv; ISDF_E_UNSUPPORTED for coulomb_sum = 1; ISDF_E_NOT_PD
 * also for S_vn or S_nn (points that make a set's C rank deficient). */
isdf_status isdf_sigma_workspace_bytes(const isdf_problem* prob, int32_t n_mu, int32_t ng,
                                       int32_t n_mu_vn, int32_t n_mu_nn, size_t* bytes);
isdf_status isdf_sigma_cohsex(isdf_handle h, const isdf_problem* prob, const void* psi,
                              const double* energies, const int32_t* mu_idx, int32_t n_mu,
                              const int32_t* mu_vn, int32_t n_mu_vn, const int32_t* mu_nn,
                              int32_t n_mu_nn, const int32_t* miller, int32_t ng,
                              void* workspace, size_t ws_bytes, void* eps_inv, double* sigma,
                              isdf_report* rep);

/* Last error message of this handle ("" if none).  Valid until the next call. */
const char* isdf_last_error(isdf_handle h);

/* Library version string. */
const char* isdf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ISDF_SMW_H */
