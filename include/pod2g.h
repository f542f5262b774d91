/*
 * pod2g.h -- C ABI of the MI355X (gfx950) POD-2G preconditioned CG library.
 *
 * The method (Nikolopoulos, Kalogeris, Stavroulakis, Papadopoulos,
 * "AI-enhanced iterative solvers for accelerating the solution of
 * large-scale parametrized systems"):
 *   - parametrised SPD finite-element systems K(theta) u = f   (Sec. 2.1, Eq. 6)
 *   - a POD basis P = Phi_r of training solutions               (Sec. 3.3, Eq. 26)
 *   - a two-grid cycle with P as prolongation, P^T as restriction,
 *     damped-Jacobi relaxation and a Galerkin coarse solve       (Sec. 2.2 Alg. 2, Eq. 30)
 *   - PCG preconditioned by one such cycle per iteration, warm-started
 *     from a surrogate prediction                               (Sec. 3.4 Alg. 3)
 *
 * Conventions (all entry points):
 *   - Array arguments are DEVICE pointers owned by the caller unless the
 *     name ends in _h (host).  The library never allocates device memory:
 *     every call that needs scratch space has a *_bytes() query and takes a
 *     caller-provided device workspace of at least that size (256-byte
 *     aligned).  Workspace contents are private to the library between the
 *     calls that share it (a pod2g_prec lives in its setup workspace).
 *   - Every call is ordered on the given HIP stream.  Calls documented as
 *     synchronous block until their stream work is done; the others are
 *     asynchronous.  Host out-parameters are written only by synchronous calls.
 *   - Every function returns an int status: 0 = POD2G_OK, negative = error.
 *     pod2g_strerror() gives a message.  No exception crosses the ABI.
 *   - No global mutable state: handles are plain structs that the caller
 *     owns; different handles may be used concurrently on different streams.
 *   - Vectors of one instance have n entries in the DOF numbering below;
 *     batched vectors are [batch][n], contiguous per instance.
 *
 * Problem family (synthetic stand-ins for the paper's Sec. 4 problems):
 *   dim = 2: plane-stress bilinear Q4 elements, unit square, N x N mesh,
 *            edge x = 0 clamped, unit traction +x on edge x = 1.
 *   dim = 3: isotropic trilinear Hex8 elements (Lame constants of Sec. 4.1),
 *            unit cube, N^3 mesh, face z = 0 clamped, unit traction +z on z = 1.
 *   Young's modulus per element, at the centroid c:
 *     E = exp(kl_scale * sum_t xi_t prod_d cos(pi a_td c_d) / (1 + sum_d a_td))
 *   with a_t the t-th multi-index of {0..3}^dim \ {0} in lexicographic order
 *   (x most significant).  Dirichlet conditions by elimination.
 *   DOF numbering: free node (i,j[,l]) has rank (i-1) + N j in 2D and
 *   i + (N+1) j + (N+1)^2 (l-1) in 3D; DOF = dim * rank + component.
 *
 * Matrix layout (block-ELL, one slot per neighbour offset in {-1,0,1}^dim,
 * slot s = (dx+1) + 3 (dy+1) [+ 9 (dz+1)], S = n_slots, H = S / 2 the
 * node's own block):
 *   colblk[s * n_nodes + node] = free-node rank of the neighbour, or the
 *     node itself for an absent neighbour;
 *   K is symmetric, so vals stores only the blocks of slots s >= H (the
 *   own block and the neighbours at a positive offset in (dz, dy, dx)
 *   order), in planes of ns = n + dim rows whose last dim rows (a "zero
 *   node") are zero:
 *     vals[((s - H) * dim + b) * ns + row] = K(row, dim * colblk[s][row / dim] + b),
 *   and a block of a slot s < H is read transposed from the neighbour j:
 *     K(dim i + r, dim j + b) = vals[((H - s) * dim + r) * ns + dim j + b]
 *   (the zero node for an absent neighbour).
 *   nvals = ns * (H + 1) * dim values per instance; batched values are
 *   [batch][nvals].
 * P is n x k column-major (column j at P + j * n), shared by all instances.
 */
#ifndef POD2G_H
#define POD2G_H

#include <stddef.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define POD2G_OK          0
#define POD2G_EINVAL     -1   /* bad argument (size, null pointer, range)   */
#define POD2G_ESIZE      -2   /* workspace smaller than the *_bytes query    */
#define POD2G_EHIP       -3   /* a HIP runtime call failed                   */
#define POD2G_ENOTSPD    -4   /* coarse matrix P^T K P: pivot <= 0           */
#define POD2G_ESMOOTHER  -5   /* omega * lambda_max(D^-1 K) >= 2 (estimate)  */
#define POD2G_EMAXIT     -6   /* iteration limit reached                     */
#define POD2G_EBREAKDOWN -7   /* p^T K p <= 0 or r^T s <= 0                   */
#define POD2G_ENAN       -8   /* non-finite residual or coefficient          */

#define POD2G_FP64   0        /* preconditioner in FP64                      */
#define POD2G_MIXED  1        /* preconditioner in FP32, outer PCG in FP64   */

#define POD2G_BETA_FR 0       /* beta = r_{k+1}^T s_{k+1} / r_k^T s_k (Alg. 3) */
#define POD2G_BETA_PR 1       /* flexible Polak-Ribiere:
                                 (r_{k+1}^T s_{k+1} - r_{k+1}^T s_k) / r_k^T s_k */

#define POD2G_MAX_K 64        /* largest coarse size k                       */

#define POD2G_SMOOTHER_JACOBI 0  /* damped Jacobi, omega (default)            */
#define POD2G_SMOOTHER_SGS    1  /* symmetric Gauss-Seidel: forward sweeps
                                    before, backward sweeps after the coarse
                                    correction, node colours (i mod 2) +
                                    2 (j mod 2) [+ 4 (l mod 2)] in turn       */

typedef struct pod2g_mesh {
  int dim;          /* 2 or 3 */
  int N;            /* elements per side, >= 1 */
  int n_terms;      /* length of xi per instance, 1..(4^dim - 1) */
  double nu;        /* Poisson ratio, 0 <= nu < 0.5 */
  double kl_scale;  /* amplitude of the log-modulus field (0.3) */
} pod2g_mesh;

typedef struct pod2g_pattern {
  pod2g_mesh mesh;
  int n_nodes;      /* free nodes */
  int n;            /* free DOFs = dim * n_nodes */
  int n_slots;      /* 3^dim */
  int n_elems;      /* N^dim */
  long long nvals;  /* stored values per instance = n * n_slots * dim */
  int *colblk;      /* device [n_slots][n_nodes], inside the pattern buffer */
  double *kref;     /* device unit-modulus element matrix, (dim 2^dim)^2,
                       row-major, element DOF dim * l + c, l = lx + 2ly + 4lz */
} pod2g_pattern;

typedef struct pod2g_prec {
  pod2g_pattern pat;
  int batch, k, nu_pre, nu_post, precision;
  double omega;
  const double *vals;   /* [batch][nvals] FP64 K (caller's) */
  const float *vals32;  /* [batch][nvals] FP32 K (caller's; MIXED only) */
  const double *dinv;   /* [batch][n] FP64 D^-1 (caller's) */
  const double *P;      /* [k][n] FP64 basis (caller's) */
  float *P32;           /* [k][n] (MIXED), in the setup workspace */
  float *dinv32;        /* [batch][n] (MIXED), in the setup workspace */
  double *KP;           /* [batch][k][n] K P, in the setup workspace */
  float *KP32;          /* [batch][k][n] FP32 K P (MIXED, 3D), in the setup workspace:
                           the cycle's first post-relaxation residual is
                           r' - (K P) e_c instead of a product with K */
  double *L;            /* [batch][k][k] row-major lower Cholesky factor of P^T K P */
  double *Linv;         /* [batch][k][k] row-major inverse of L (lower triangular):
                           the cycle's coarse solve is e_c = Linv^T (Linv r_c) */
  double *lam;          /* [batch] power-iteration estimate of lambda_max(D^-1 K) */
  int *status;          /* [batch] per-instance setup status (device) */
  void *work;           /* the setup workspace this handle lives in */
  int smoother;         /* POD2G_SMOOTHER_*; pod2g_setup sets JACOBI */
} pod2g_prec;

const char *pod2g_strerror(int status);

/* ---- pattern ------------------------------------------------------------
 * Builds the free-DOF map, the block-ELL column indices and the unit-modulus
 * element matrix (2^dim-point Gauss quadrature) of Sec. 2.1 Eq. 5.
 * dbuf: device buffer of pod2g_pattern_bytes(mesh) bytes that holds colblk
 * and kref for the lifetime of *out.  Asynchronous.
 * Errors: EINVAL (mesh out of range, n >= 2^31 / 81), ESIZE.                */
size_t pod2g_pattern_bytes(const pod2g_mesh *mesh);
int pod2g_pattern_build(const pod2g_mesh *mesh, void *dbuf, size_t bytes,
                        pod2g_pattern *out, hipStream_t stream);

/* ---- assembly (Sec. 2.1, Eqs. 5-6) ---------------------------------------
 * For each of `batch` instances b with field coefficients xi[b * n_terms ..]
 * (device, FP64): element moduli E_e, then every stored value of
 * K = sum_e E_e A_e^T K_ref A_e restricted to free DOFs, gathered per stored
 * entry (deterministic, no atomics); D^-1 = 1/diag(K).  Optional outputs may
 * be NULL: vals32 (FP32 copy of vals, RNE), f (the load vector, [n], the
 * same for every instance).  Asynchronous.  Errors: EINVAL, ESIZE.          */
size_t pod2g_assemble_bytes(const pod2g_pattern *pat, int batch);
int pod2g_assemble(const pod2g_pattern *pat, const double *xi, int batch,
                   double *vals, float *vals32, double *dinv, double *f,
                   void *work, size_t bytes, hipStream_t stream);

/* ---- preconditioner setup (Alg. 2 restrict-and-solve step, Eq. 28) -------
 * Per instance: KP = K P, K_c = P^T (K P) (k x k), its FP64 Cholesky factor
 * L (pivot <= 0 -> POD2G_ENOTSPD in status[b]); with power_iters > 0 also a
 * power-iteration estimate of lambda_max(D^-1 K) from the all-ones vector
 * (omega * lambda >= 2 -> POD2G_ESMOOTHER).  MIXED also makes FP32 copies of
 * P and D^-1.  k = 0 gives the smoother-only cycle.  P must be 16-byte
 * aligned (EINVAL otherwise; any torch or hipMalloc allocation is).  vals32 may be NULL for
 * FP64.  The handle *out points into work, which must outlive it.
 * Asynchronous: per-instance errors land in out->status and are reported by
 * pcg_solve / pod2g_setup_status.  Returns EINVAL/ESIZE/EHIP synchronously. */
size_t pod2g_setup_bytes(const pod2g_pattern *pat, int k, int batch, int precision);
int pod2g_setup(const pod2g_pattern *pat, const double *vals, const float *vals32,
                const double *dinv, const double *P, int k, double omega,
                int nu_pre, int nu_post, int precision, int batch, int power_iters,
                void *work, size_t bytes, pod2g_prec *out, hipStream_t stream);
/* Selects the relaxation of the cycle (Sec. 2.2: the relaxation slot of
 * Alg. 2; Gauss-Seidel is the paper's own form): POD2G_SMOOTHER_JACOBI or
 * POD2G_SMOOTHER_SGS.  The Jacobi stability guard of pod2g_setup concerns
 * damped Jacobi only.  Host-only.  Errors: EINVAL.                          */
int pod2g_set_smoother(pod2g_prec *prec, int smoother);
/* Redoes the setup of instance `slot` of an existing handle, in place, from
 * that instance's current vals / dinv (after the caller re-assembled it):
 * K P, K_c, L, Linv, status, lambda estimate and the FP32 D^-1.  The shared
 * FP32 basis and the other instances are left alone.  Asynchronous.
 * Errors: EINVAL (slot out of range, handle without workspace), EHIP.      */
int pod2g_setup_slot(const pod2g_prec *prec, int slot, int power_iters, hipStream_t stream);
/* Synchronous: copies the per-instance setup status (and, if lam_h is not
 * NULL, the lambda_max estimates) to host arrays of length batch.          */
int pod2g_setup_status(const pod2g_prec *prec, int *status_h, double *lam_h,
                       hipStream_t stream);

/* ---- one two-grid cycle (Alg. 3 preconditioning steps; Alg. 2 body) -------
 * s = B r for every instance: nu_pre damped-Jacobi sweeps from x = 0,
 * r' = r - K x, r_c = P^T r', L L^T e_c = r_c, x += P e_c, nu_post sweeps.
 * r, s: [batch][n].  Asynchronous.                                          */
size_t pod2g_apply_bytes(const pod2g_prec *prec);
int pod2g_apply(const pod2g_prec *prec, const double *r, double *s,
                void *work, size_t bytes, hipStream_t stream);

/* ---- one cycle without allocation or workspace -----------------------------
 * For callers that cannot allocate device memory or pass a workspace: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  pod2g_apply without the workspace: the cycle runs in a scratch
 * array of POD2G_NOALLOC_SCRATCH_BYTES that the library holds on every GPU
 * it runs on until the process ends (the GPU current at the call, which must
 * be the stream's; the first call on a GPU looks the array's address up,
 * so make it outside stream capture).  Nothing is allocated.  Every call on
 * one GPU shares that GPU's array, which keeps the last call's contents (a
 * call clears the state it needs itself): calls in order on one stream are
 * safe, calls that overlap on one GPU (several streams or host threads)
 * race and give wrong results.  Asynchronous.  Errors: EINVAL, EHIP, and
 * ESIZE when pod2g_apply_bytes(prec) exceeds the array (FP64: about 1e6
 * unknowns x instances).                                                   */
#define POD2G_NOALLOC_SCRATCH_BYTES (64 * 1024 * 1024)
int pod2g_apply_noalloc(const pod2g_prec *prec, const double *r, double *s,
                        hipStream_t stream);

/* ---- PCG (Sec. 3.4 Alg. 3; Sec. 2.1 Alg. 1 when prec == NULL) ------------
 * Solves K_b u_b = f for b < batch from the initial guesses in u (overwritten
 * by the solutions).  Stops when ||r|| <= rtol ||f|| on the recursive
 * residual, then checks the true residual f - K u; on a gap the true residual
 * replaces r and CG restarts from it.  maxit bounds the completed updates.
 * beta: POD2G_BETA_FR or POD2G_BETA_PR.  f: [n] shared by all instances.
 * Synchronous.  Host outputs (length batch, each may be NULL): iters_h =
 * completed iterations, relres_h = true ||f - K u|| / ||f|| at exit,
 * status_h = per-instance status.  Returns POD2G_OK if every instance
 * converged, else the first failing instance's status.                     */
size_t pcg_solve_bytes(const pod2g_pattern *pat, int batch, int k, int precision);
int pcg_solve(const pod2g_pattern *pat, const double *vals, int batch,
              const pod2g_prec *prec, const double *f, double *u,
              double rtol, int maxit, int beta,
              int *iters_h, double *relres_h, int *status_h,
              void *work, size_t bytes, hipStream_t stream);

/* ---- standalone two-grid solver (Sec. 3.3 scheme iterated on its own) ----
 * u_b <- u_b + B_b (f - K_b u_b) (the cycle of pod2g_apply, error operator
 * of Eq. 30) from the initial guesses in u until ||f - K u|| <= rtol ||f||
 * or maxit (>= 1) cycles, as the POD-2G solver is used on its own in the
 * Sec. 4 comparisons.  prec is required.  Workspace: pcg_solve_bytes.
 * Synchronous; outputs as pcg_solve (relres_h is the true residual: the
 * iteration recomputes it every cycle).  Returns OK, EMAXIT or ENAN (first
 * failing instance), EINVAL, ESIZE, EHIP.                                   */
int pod2g_stationary_solve(const pod2g_pattern *pat, const double *vals, int batch,
                           const pod2g_prec *prec, const double *f, double *u,
                           double rtol, int maxit, int *iters_h, double *relres_h,
                           int *status_h, void *work, size_t bytes, hipStream_t stream);

/* ---- reduced-order (POD-Galerkin) solution as a warm start -----------------
 * u_b = P (P^T K_b P)^{-1} P^T f (Sec. 3.3, the reduced system of the POD
 * basis and its lift): the coarse factor of the setup applied to the
 * restricted load, prolonged.  A surrogate-free initial guess for pcg_solve.
 * FP64.  u: [batch][n] (overwritten).  work: pod2g_rom_bytes(prec) bytes.
 * Asynchronous.  Errors: EINVAL (no basis: k = 0), ESIZE.                   */
size_t pod2g_rom_bytes(const pod2g_prec *prec);
int pod2g_rom_start(const pod2g_prec *prec, const double *f, double *u, void *work,
                    size_t bytes, hipStream_t stream);

/* ---- live kernel timing ----------------------------------------------------
 * A timer holds per_call pairs of HIP events (created by pod2g_timer_create,
 * released by pod2g_timer_destroy).  In the second chunk of iterations of a
 * timed solve, the first per_call launches of the selected kernel go through
 * hipExtLaunchKernel, whose events receive the dispatch's own start and end
 * timestamps; if every instance was still iterating through that chunk,
 * their durations are added to total_ms / launches.  A timed plan solve runs
 * that chunk as individual launches (same kernels, same results) and the
 * others as graph replays.  Kernel ids:                                     */
#define POD2G_TK_SPMV_PQ     1   /* q = K p with p^T q (outer SpMV)            */
#define POD2G_TK_SWEEP       2   /* damped-Jacobi sweep inside the cycle       */
#define POD2G_TK_SWEEP_FINAL 3   /* last post-sweep with r^T s                 */
#define POD2G_TK_RESTRICT    4   /* residual + restriction + coarse solve      */
#define POD2G_TK_PROLONG     5   /* prolongation and correction                */
#define POD2G_TK_UPDATE      6   /* u, r updates with ||r||^2                  */

typedef struct pod2g_timer {
  int kernel;        /* POD2G_TK_* */
  int per_call;      /* event pairs = launches timed per solve */
  hipEvent_t *start, *stop;   /* host arrays of events, owned by the timer */
  double total_ms;   /* accumulated kernel time */
  long long launches;/* accumulated timed launches */
} pod2g_timer;

int pod2g_timer_create(int kernel, int per_call, pod2g_timer *out);
int pod2g_timer_reset(pod2g_timer *t);      /* zeroes total_ms and launches */
int pod2g_timer_destroy(pod2g_timer *t);
/* pcg_solve with a timer (NULL: identical to pcg_solve).                    */
int pcg_solve_timed(const pod2g_pattern *pat, const double *vals, int batch,
                    const pod2g_prec *prec, const double *f, double *u,
                    double rtol, int maxit, int beta,
                    int *iters_h, double *relres_h, int *status_h,
                    void *work, size_t bytes, pod2g_timer *timer, hipStream_t stream);

/* ---- captured solve plans ---------------------------------------------------
 * A plan captures `chunk` PCG iterations on fixed buffers (the arguments of
 * pcg_solve: pattern, values, preconditioner workspace, f, u, solve
 * workspace) into one HIP graph; pcg_plan_solve then runs the solve like
 * pcg_solve but launches that graph once per chunk instead of the
 * individual kernels, and checks convergence between chunks.  The plan
 * stays valid while those buffers live and keep their sizes; their contents
 * may change between solves (new theta, new warm start, new setup in the
 * same setup workspace).  With a timer (which must outlive the plan), the
 * second chunk of every solve is timed as described above.  pcg_plan_solve is synchronous
 * and has pcg_solve's outputs and statuses.  An odd chunk is rounded up to
 * the next even number.  Plans are host objects: create, solve and destroy
 * them from one thread.                                                     */
typedef struct pod2g_plan pod2g_plan;
int pcg_plan_create(const pod2g_pattern *pat, const double *vals, int batch,
                    const pod2g_prec *prec, const double *f, double *u, int chunk,
                    void *work, size_t bytes, pod2g_timer *timer, pod2g_plan **out);
int pcg_plan_solve(pod2g_plan *plan, double rtol, int maxit, int beta,
                   int *iters_h, double *relres_h, int *status_h, hipStream_t stream);
int pcg_plan_destroy(pod2g_plan *plan);

/* Launch-parameter tuning of a plan on its own buffers: times `trials`
 * (2..1000) PCG iterations from a fresh start for each candidate value of
 * one parameter at a time and keeps the fastest, then recaptures the plan:
 * the workgroups of the batched restriction (256..2048, batched FP32 cycle
 * only), the direction update folded into the outer SpMV or run as its own
 * pass, the vector update fused with the second Jacobi pre-relaxation
 * sweep or not, the scalar sums r^T s and p^T q finished by the kernels that read
 * them (each workgroup re-reads the partials) or by the producer's last
 * workgroup, the neighbourhood of each 2D node block staged in LDS or
 * gathered from the caches, the row groups of the batched restriction loaded together
 * (1, 2, 4), and the instance grouping of the node-wise block order
 * (divisors of the batch up to 8).  It overwrites u and the solve workspace: call it
 * before loading the initial guess.  Synchronous.  out may be NULL.       */
typedef struct pod2g_tuning {
  int bgrid;               /* workgroups of the batched restriction */
  int fuse_dir;            /* 1: p = s + beta p formed inside the outer SpMV */
  int igroup;              /* instances per group in the node-wise block order */
  int xwin;                /* > 0: 2D node blocks gather x from LDS (+- xwin nodes staged) */
  int cons;                /* 1: r^T s and p^T q summed by every workgroup of their consumers */
  int fuse_upd;            /* 1: vector update fused with the second pre-relaxation sweep */
  int ptr_grp;             /* 1, 2 or 4: 16-row groups of the batched restriction's MFMA
                              contraction loaded together per wave iteration */
  float ms_per_iteration;  /* time of one iteration with the chosen values */
} pod2g_tuning;
int pcg_plan_tune(pod2g_plan *plan, int trials, pod2g_tuning *out, hipStream_t stream);

/* Set a plan's launch parameters explicitly (for instance values an earlier
 * pcg_plan_tune chose) and recapture it; pcg_plan_config reads them
 * (ms_per_iteration = 0).  bgrid in 1..min(workgroups of n rows, 2048);
 * fuse_dir, cons and fuse_upd 0 or 1; igroup a divisor of the batch up to
 * 8; xwin 0, or positive for LDS staging (2D only: the library sets the
 * window); ptr_grp 1, 2 or 4; ms_per_iteration is ignored.  Anything else: POD2G_EINVAL and
 * the plan is unchanged.  Only bgrid (the partition of the batched
 * restriction's sums) and fuse_upd (the grouping of the ||r||^2 and
 * r^T s_old partials) change rounding; the other parameters give the same
 * bits.  Not thread-safe with a solve on the same plan.                   */
int pcg_plan_configure(pod2g_plan *plan, const pod2g_tuning *cfg);
int pcg_plan_config(const pod2g_plan *plan, pod2g_tuning *out);

/* ---- served solves (continuous batching over slot groups) -----------------
 * Many independent queries theta (Sec. 3, the multi-query setting) arrive
 * over time.  A server owns n_groups slot groups; group g is one problem
 * class: one pattern, one basis P and prec->batch slots, each slot holding
 * one query's K, D^-1, coarse factor (the preconditioner handle's arrays),
 * u and CG state (the group's solve workspace, pcg_solve_bytes(pat,
 * prec->batch, prec->k, prec->precision) bytes).  The caller writes a
 * query into a free slot (pod2g_assemble on the slot's rows with batch 1,
 * pod2g_setup_slot, u_slot = x0) and calls pod2g_server_admit.
 * pod2g_serve_step launches one HIP graph that advances every live slot of
 * every group by `chunk` PCG iterations (Alg. 3, the same kernels and
 * arithmetic as pcg_solve with batch = prec->batch), forms the true
 * residual of the admitted and the stopped slots, and either finishes a
 * slot or restarts it from its true residual (the exit check of pcg_solve).
 * It then copies one pod2g_slot_info per slot (groups in order, slots in
 * order) to info_h; done = 1 marks a finished solve whose u is final.
 * Steps are asynchronous: synchronize the stream before reading info_h
 * (pinned host memory keeps the copy asynchronous).  A slot's result is
 * bitwise the one pcg_solve gives for it in a batch of the same size,
 * whatever the other slots hold.  All calls of one server go to one stream
 * from one host thread.  Errors: EINVAL, ESIZE, EHIP.                      */
typedef struct pod2g_slot_info {
  int done;        /* 1: solve finished (or slot free), 0: running */
  int iter;        /* completed PCG iterations */
  int status;      /* POD2G_OK, EMAXIT, EBREAKDOWN, ENAN or the setup error */
  int pad;
  double relres;   /* true ||f - K u|| / ||f|| of the final iterate */
} pod2g_slot_info;

typedef struct pod2g_group {
  const pod2g_pattern *pat;
  const double *vals;     /* [batch][nvals], the handle's vals */
  const pod2g_prec *prec; /* batch = slots of the group (required) */
  const double *f;        /* [n] */
  double *u;              /* [batch][n] */
  void *work;             /* solve workspace of the group */
  size_t bytes;
} pod2g_group;

typedef struct pod2g_server pod2g_server;
/* Captures the step graph; every slot starts free.  chunk >= 2, even
 * (an odd chunk is rounded up).  The groups' buffers must outlive the
 * server and keep their addresses.                                        */
int pod2g_server_create(const pod2g_group *groups, int n_groups, int chunk,
                        pod2g_server **out, hipStream_t stream);
/* Starts the solve of slot `slot` of group `group` from u_slot = x0 with
 * tolerance rtol, iteration limit maxit and beta kind; a slot whose setup
 * failed finishes at the next step with that setup status.  The slot must
 * not be running.  Asynchronous.                                           */
int pod2g_server_admit(pod2g_server *srv, int group, int slot, double rtol, int maxit,
                       int beta, hipStream_t stream);
int pod2g_serve_step(pod2g_server *srv, pod2g_slot_info *info_h, hipStream_t stream);
/* The step of one group alone (its own graph) with the copy of that group's
 * slot outcomes into its part of info_h: groups stepped on different streams
 * advance at their own pace, so a small class is not held to the iteration
 * rate of a large one.  A group must not be stepped on two streams at once.
 * Asynchronous.                                                            */
int pod2g_serve_step_group(pod2g_server *srv, int group, pod2g_slot_info *info_h,
                           hipStream_t stream);
/* pod2g_serve_step_group over the group's first slots only: the step graph
 * of the smallest captured prefix (4, 8, 16, ... slots, else the whole
 * group) that holds slots 0 .. nslots - 1, so free slots past the last live
 * one cost no launches.  Slots at or past the prefix must not be running
 * (they do not advance).  A slot gets the same bits from any prefix.
 * Asynchronous.  Errors: EINVAL (nslots outside 0 .. group slots), EHIP.   */
int pod2g_serve_step_prefix(pod2g_server *srv, int group, int nslots,
                            pod2g_slot_info *info_h, hipStream_t stream);
int pod2g_server_slots(const pod2g_server *srv);   /* total slots, or EINVAL */
/* A HIP stream (default priority) whose kernels run only on compute units
 * cu_first .. cu_first + cu_count - 1 of the current GPU, in the runtime's
 * CU-mask numbering: a serving loop can give each problem class its own
 * share of the GPU, so that the small, latency-bound kernels of one class do
 * not wait for compute units behind the large kernels of another.  Release
 * with pod2g_stream_destroy once nothing refers to the stream any more (no
 * pending work, no runtime or framework object that recorded an event on
 * it; a serving process keeps such streams to the end).  Errors: EINVAL
 * (range outside the GPU's compute units), EHIP.                           */
int pod2g_stream_create_cus(int cu_first, int cu_count, hipStream_t *out);
int pod2g_stream_destroy(hipStream_t stream);
int pod2g_server_destroy(pod2g_server *srv);

/* ---- profiling markers -------------------------------------------------------
 * Launches an empty one-thread kernel named k_mark_begin (which = 0) or
 * k_mark_end (which = 1) on the stream, so that a kernel trace can be cut
 * to the dispatches between them.  Asynchronous.                            */
int pod2g_mark(int which, hipStream_t stream);

/* ---- single kernels (measurement and parity checks) ---------------------
 * y_b = K_b x_b (FP64).  Asynchronous.                                      */
int pod2g_spmv(const pod2g_pattern *pat, const double *vals, int batch,
               const double *x, double *y, hipStream_t stream);
/* nsweeps damped-Jacobi sweeps x <- x + omega D^-1 (b - K x) (the relaxation
 * of Alg. 2) in place on x, using tmp ([batch][n]) as the second buffer;
 * the same kernel as the cycle's sweeps.  Asynchronous.                     */
int pod2g_jacobi(const pod2g_pattern *pat, const double *vals, const double *dinv,
                 int batch, double omega, int nsweeps, const double *b, double *x,
                 double *tmp, hipStream_t stream);

/* nsweeps Gauss-Seidel sweeps on K x = b in place on x (FP64), in the
 * multicolour order of POD2G_SMOOTHER_SGS, forward or (backward != 0)
 * reversed: the same kernels as the cycle's sweeps.  Asynchronous.          */
int pod2g_gauss_seidel(const pod2g_pattern *pat, const double *vals, const double *dinv,
                       int batch, int nsweeps, int backward, const double *b, double *x,
                       hipStream_t stream);

/* ---- offline POD (Sec. 3.3, steps 1-2) ----------------------------------
 * From N snapshots U ([N][n], one solution per row block), the Gram matrix
 * G = U^T U, its eigenpairs by cyclic Jacobi rotations, and
 * P = U Psi_k Lambda_k^{-1/2} (Eq. 26) with the k largest eigenvalues.
 * lam: [N] all eigenvalues, descending (device).  N <= 256, k <= min(N, 64).
 * Rank below k (lambda_k <= N eps lambda_1) -> POD2G_EINVAL.  Synchronous.  */
size_t pod2g_pod_basis_bytes(int n, int N, int k);
int pod2g_pod_basis(const double *U, int n, int N, int k, double *P, double *lam,
                    void *work, size_t bytes, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* POD2G_H */
