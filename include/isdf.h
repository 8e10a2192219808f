/*
 * isdf.h -- C ABI of the MI355X (gfx950) k-point ISDF library.
 *
 * The library evaluates, on one GPU, the hot path of translational-symmetry
 * adapted interpolative separable density fitting (k-point FFTISDF):
 *
 *   isdf_create          orbitals phi^k_mu(r) on the unit-cell grid plus the
 *                        interpolation points r_I (section "Periodic k-point
 *                        FFTISDF representation of integrals", eq. (1)-(2));
 *   isdf_fit             interpolating vectors X^k, metric Pi^q (eq. (4)),
 *                        right-hand side eta^q (eq. (5)), both as convolutions
 *                        over k (Algorithm 1), and the FP64 pivoted Cholesky
 *                        factor of every Pi^q (the solve of eq. (3));
 *   isdf_coulomb_kernel  W^q from V^q = Coulomb(eta^q) and Pi W Pi = V
 *                        (eqs. (6)-(8)), grid FFTs with the 4 pi/|G+q|^2 kernel;
 *   isdf_fragment_eri    fragment ERIs from W^q and fragment coefficients
 *                        C^k_{mu p} (eqs. (17), (19)-(20), Algorithm 2);
 *   isdf_submit/poll     the same as served requests (continuous batching);
 *   isdf_graph_*         one fragment batch captured as a HIP graph and replayed;
 *   isdf_autotune        launch tiling of the fragment contraction timed on a
 *                        caller's batch (isdf_set_tiling sets it directly).
 *
 * Conventions (the paper leaves them implicit; they are fixed here):
 *   - complex numbers are interleaved (re, im) float64 pairs ("c128");
 *   - lattice rows a1, a2, a3 in bohr; grid index i = (i1*n2 + i2)*n3 + i3 is
 *     the point (i1/n1) a1 + (i2/n2) a2 + (i3/n3) a3;
 *   - the k mesh is Gamma-centred, k index = (j1*m2 + j2)*m3 + j3 is the point
 *     sum_d (j_d/m_d) b_d; q is the mesh difference of pair momenta (mod m),
 *     wrapped to [-1/2, 1/2) per axis inside the Coulomb kernel; each DFT
 *     index of the grid stands for K = G + q at its representative nearest
 *     zero per axis (|K_d| <= n_d/2 in units of b_d, the kernel averaged over
 *     the two representatives at a tie K_d = +-n_d/2), and the K = 0 term is
 *     dropped;
 *   - a superscript -k in the paper is read as the complex conjugate at k;
 *   - ERIs are in Hartree, chemists' notation with the conjugate on p and r:
 *       (pq|rs) = int int conj(psi_p) psi_q (x) conj(psi_r) psi_s (y) / |x-y|,
 *     psi_p = N_k^{-1/2} sum_k sum_mu C^k_{mu p} phi^k_mu (eq. (17)), output
 *     layout [p][q][r][s] C order (the paper's V_pqrs is (qp|sr) here).
 *
 * Every call returns an isdf_status; 0 is success.  Calls never abort and
 * never throw; on failure the context records a message that
 * isdf_last_error() returns.  A context is used by one host thread at a time,
 * except isdf_submit / isdf_poll / isdf_cancel, which are thread-safe.
 */
#ifndef ISDF_H
#define ISDF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct isdf_ctx_s* isdf_ctx;

typedef enum {
  ISDF_OK = 0,
  ISDF_E_INVALID = -1,   /* bad argument (null pointer, size, layout)           */
  ISDF_E_NOMEM = -2,     /* memory planner or device allocation refused         */
  ISDF_E_STATE = -3,     /* call out of order (e.g. ERIs before the kernel)     */
  ISDF_E_NUMERIC = -4,   /* Cholesky breakdown, non-finite value (q in message) */
  ISDF_E_DEVICE = -5,    /* HIP runtime error                                   */
  ISDF_E_BUSY = -6,      /* request queue full                                  */
  ISDF_E_NOTFOUND = -7,  /* unknown ticket                                      */
  ISDF_E_CANCELLED = -8  /* request was cancelled                               */
} isdf_status;

typedef enum {
  ISDF_FP64 = 0,        /* every GEMM in FP64 MFMA                                 */
  ISDF_MIXED_FP32 = 1,  /* the fragment GEMMs (U^q = R^q W^q and the contraction)
                           in FP32 MFMA, FP32 accumulation within one class of q
                           (or one K segment), FP64 across them; the fit and the
                           Coulomb kernel stay FP64                              */
  ISDF_MIXED_BF16X3 = 2, /* the same GEMMs with operands split hi+lo in bf16 and
                           three bf16 MFMA products (hi*hi + hi*lo + lo*hi)     */
  ISDF_MIXED_BF16 = 3   /* the same GEMMs with operands rounded to bf16, one bf16
                           MFMA per real product, no split correction: error
                           measured at 3e-4 to 2e-2 of the largest ERI, so
                           within 1e-6 Eh only where the ERIs are small (a
                           1000-k cell with max |V| 1.6e-5 Eh: 4.5e-8 Eh);
                           callers check their own bound                     */
} isdf_precision;

/* flags for isdf_create */
#define ISDF_INPUT_DEVICE 0x1u   /* orbitals / ip_index are device pointers      */
#define ISDF_NO_PIVOT 0x2u       /* plain Cholesky: a singular Pi^q is an error  */
/* isdf_coulomb_kernel takes the zeta route of eqs. (3) and (6) (xi^q = Pi^{q+}
 * eta^q, FFT, W^q = xihat^H c xihat) instead of eqs. (7)-(8) */
#define ISDF_ZETA_ROUTE 0x4u
/* the mixed fragment GEMMs keep U^q = R^q W^q (no factor form, below) */
#define ISDF_W_PLAIN 0x8u
/* at most n classes {q, -q} of eta per q batch (bits 16-31; 0 = as many as
 * fit, see isdf_fit) */
#define ISDF_Q_BATCH(n) ((((uint32_t)(n)) & 0xFFFFu) << 16)

/* request states reported by isdf_poll */
#define ISDF_REQ_QUEUED 0
#define ISDF_REQ_RUNNING 1
#define ISDF_REQ_DONE 2
#define ISDF_REQ_FAILED 3
#define ISDF_REQ_CANCELLED 4

/* fragment buffers: C and eri are device pointers when this bit is set in
 * isdf_fragment_eri's flags / isdf_request.flags, host pointers otherwise */
#define ISDF_FRAG_DEVICE 0x1u
/* isdf_fragment_eri flags bits 8-15: run every fragment alone with its n_f^2
 * pairs in n blocks (at most n_f^2; 0 or 1 = blocks only where memory
 * requires them) */
#define ISDF_FRAG_BLOCKS(n) ((((uint32_t)(n)) & 0xFFu) << 8)

/*
 * Create a context (eq. (1)-(2) inputs).
 *   lattice   [3][3] float64, rows a1 a2 a3 (bohr), host memory.
 *   grid      [3] grid points per axis (each 2..64, factorisable into 2,3,5,7).
 *   kmesh     [3] k points per axis (each 1..16).
 *   n_orb     orbitals per k point (1..256).
 *   orbitals  c128 [N_k][n_orb][N_g], host or device (ISDF_INPUT_DEVICE).
 *   ip_index  int32 [n_ip] grid indices r_I (0 <= r_I < N_g, distinct), caller
 *             selected (the paper selects them by pivoted Cholesky).
 *   n_ip      number of interpolation points (1..2048).
 *   hip_stream  hipStream_t every call of this context launches on (0 = null
 *               stream); the caller keeps it alive until isdf_destroy.
 * The library copies orbitals and ip_index into its own device memory; the
 * caller may free them on return.  Error: ISDF_E_INVALID, ISDF_E_NOMEM,
 * ISDF_E_DEVICE; *out is NULL on failure.
 */
isdf_status isdf_create(isdf_ctx* out, const double* lattice, const int32_t grid[3],
                        const int32_t kmesh[3], int32_t n_orb, const void* orbitals,
                        const int32_t* ip_index, int32_t n_ip, uint32_t flags,
                        void* hip_stream);

/*
 * Interpolation points by pivoted Cholesky of the pair products (the
 * IP-selection paragraph of the section "Periodic k-point FFTISDF
 * representation of integrals"): the products
 * phi^{k_mu}_mu(r) conj(phi^{k_nu}_nu(r)) have the Gram matrix
 * M(x, y) = |sum_k sum_mu phi^k_mu(x) conj(phi^k_mu(y))|^2 over grid points,
 * and the greedy Cholesky of M with diagonal pivoting selects its first n_ip
 * pivots: start from the residual d(x) = M(x, x) = rho(x)^2; at each step take
 * the point p of largest residual (lowest index among equals), form the
 * factor column L(x) = (M(x, p) - sum of the previous columns' L(x) L(p)) /
 * sqrt(d(p)), lower d by L(x)^2 and set d(p) = 0.  M is never formed: a step
 * reads the orbitals once.  FP64.
 *   grid, kmesh, n_orb  as isdf_create (n_ip <= N_g).
 *   orbitals   c128 [N_k][n_orb][N_g], host or device (ISDF_INPUT_DEVICE),
 *              the layout isdf_create takes.
 *   ip_out     int32 [n_ip], host: the pivots in selection order, ready to
 *              pass to isdf_create as ip_index.
 *   residual_out  float64 [n_ip], host, or NULL: the residual d(p) of each
 *              pivot when it was chosen (non-increasing in exact arithmetic;
 *              its decay measures how well the first i points span the pair
 *              products).
 *   hip_stream  stream of the launches (0 = null stream).
 * Synchronous; device workspace n_ip N_g 8 bytes plus a few grid-sized
 * vectors (and a copy of host orbitals), freed on return.  Errors
 * (message from isdf_last_error(NULL)): ISDF_E_INVALID for bad sizes or
 * pointers; ISDF_E_NUMERIC when a step's largest residual is not positive
 * (the products span fewer than n_ip grid columns, or the orbitals are not
 * finite): ip_out / residual_out then hold the pivots found before it and -1
 * / 0 after; ISDF_E_NOMEM, ISDF_E_DEVICE.
 */
isdf_status isdf_select_points(const int32_t grid[3], const int32_t kmesh[3], int32_t n_orb,
                               const void* orbitals, int32_t n_ip, int32_t* ip_out,
                               double* residual_out, uint32_t flags, void* hip_stream);

/*
 * The fit: X^k_{I mu} = phi^k_mu(r_I); T^k = X^k X^{k H}; Pi^q by the k
 * convolution of Algorithm 1 (|FFT_k^{-1} T|^2, FFT_k); eta^q_I(r) by the same
 * convolution of T^k_I(r) = sum_mu X^k_{I mu} conj(phi^k_mu(r)), on tiles of
 * grid points and interpolation points of about 1 GiB each (the environment
 * variable ISDF_RHS_TILE_BYTES, read by isdf_create, sets another size; the
 * result does not depend on it; isdf_stats reports r_tile and ip_tile); then
 * the FP64 Cholesky factor of every Pi^q with diagonal pivoting (relative
 * tolerance 1e-13; the rank is reported by isdf_stats).  Synchronous.
 * Pi^{-q}, eta^{-q} and W^{-q} are the complex conjugates of those at q, so
 * one q of each class {q, -q} is computed and stored.  eta of every class
 * is formed here when it fits in 60 % of the device memory left after the
 * context's other buffers (capped by ISDF_Q_BATCH); otherwise
 * isdf_coulomb_kernel forms it per q batch, isdf_get_rhs is unavailable, and
 * the kernel hands the fit's transient buffers (eta, the RHS tiles, T^k of
 * the metric, the factorisation scratch) back to the fragment workspaces
 * when it ends (the next fit allocates them again).  Everything here is
 * FP64 in every precision; `prec` is accepted for symmetry with
 * isdf_coulomb_kernel.  Error: ISDF_E_INVALID for an unknown precision;
 * ISDF_E_NUMERIC when ISDF_NO_PIVOT is set and a Pi^q is singular.
 */
isdf_status isdf_fit(isdf_ctx ctx, isdf_precision prec);

/*
 * W^q for all q (eqs. (6)-(8)): grid FFT of eta^q(r) exp(-i q.r), scaled by
 * sqrt(Omega 4 pi/|K|^2)/N_g (FP64; K the representative of G+q nearest
 * zero per axis, the kernel averaged over the two at a tie +-n/2),
 * V^q = eta~ eta~^H (FP64 MFMA), W^q = Pi^{q+} V^q Pi^{q+} by FP64
 * triangular solves with the factor of isdf_fit; one q per class {q, -q},
 * in q batches (eta formed per batch) when isdf_fit did not form eta.
 * The kernel is FP64 in every precision: W^q amplifies the rounding of eta
 * and V^q by up to cond(Pi^q) on each side, and at the conditioning of the
 * workloads (cond(Pi^q) 1e4-5e5) an FP32 or bf16 hi+lo V^q moves the ERIs by
 * 3e-6 to 2e-5 Eh; the mixed precisions apply to the fragment GEMMs, where
 * the error with an FP64 W^q stays within the 1e-6 Eh bound.  `prec` is
 * accepted for symmetry with isdf_fragment_eri.
 * Consumes eta (isdf_get_rhs is invalid afterwards).  Synchronous.
 * With ISDF_ZETA_ROUTE (isdf_create flags) the kernel follows eqs. (3) and
 * (6) instead: xi^q = Pi^{q+} eta^q for every grid point (one FP64 MFMA
 * product per class with the pseudo-inverse P G P^T of the pivoted factor),
 * the same scaled grid FFT of xi^q(r) exp(-i q.r), and W^q = xi~ xi~^H
 * directly (FP64 MFMA); W^q equals the default route's in exact arithmetic.
 * It needs eta of every class resident (isdf_fit formed it) and a second
 * eta-sized buffer for xi (freed on return), else ISDF_E_NOMEM; eta stays
 * valid.
 * Error: ISDF_E_STATE before isdf_fit.
 */
isdf_status isdf_coulomb_kernel(isdf_ctx ctx, isdf_precision prec);

/* Test hooks: copy Pi^q / W^q (c128 [n_ip][n_ip]) or X^k (c128 [n_ip][n_orb])
 * to host memory `out`.  Error: ISDF_E_STATE if not computed yet,
 * ISDF_E_INVALID for q or k out of range. */
isdf_status isdf_get_metric(isdf_ctx ctx, int32_t q, void* out);
isdf_status isdf_get_kernel(isdf_ctx ctx, int32_t q, void* out);
isdf_status isdf_get_ivs(isdf_ctx ctx, int32_t k, void* out);
/* Copy eta^q (c128 [n_ip][N_g]) to host; valid between isdf_fit and
 * isdf_coulomb_kernel (and only when the fit formed eta of every class). */
isdf_status isdf_get_rhs(isdf_ctx ctx, int32_t q, void* out);
/* Test hook: copy the Coulomb-weighted transform of eq. (7),
 *   eta~^q_I(G) = sqrt(Omega 4 pi / |K|^2) / N_g sum_r eta^q_I(r) exp(-i (G+q).r)
 * (K as in isdf_coulomb_kernel; 0 at K = 0), as it enters V^q = eta~ eta~^H
 * (FP64).  out: host c128 [n_ip][N_g], G in the
 * FFT order of the grid (index i_d stands for G_d = i_d wrapped to
 * [-n_d/2, n_d/2)).  Valid after isdf_coulomb_kernel until the next isdf_fit.
 * Error: ISDF_E_STATE before isdf_coulomb_kernel or after one that ran in q
 * batches, ISDF_E_INVALID for a bad q. */
isdf_status isdf_get_eta_tilde(isdf_ctx ctx, int32_t q, void* out);

/*
 * Fragment ERIs for a batch of fragments in one pass (eqs. (19)-(20),
 * Algorithm 2): T^k = X^k C^k, k -> R transform, outer products, R -> q
 * transform giving R^q_{I,pq}, U^q = W^q R^q, then the Hermitian contraction
 * sum_q R^{q H}-weighted products accumulated over q (FP64 accumulation across
 * q in every precision), one grouped persistent launch for all fragments.
 * Factor form (mixed precisions): isdf_coulomb_kernel also factors every
 * W^q = L L^H (FP64, no pivoting); when every pivot is above 1e-13 of its
 * matrix's largest diagonal entry (isdf_stats: "w_factor"), the mixed paths
 * form Y^q = R^q L^q (a triangular product: half the work of U^q) and the
 * contraction sum_q Y^q Y^{qH} (same ERIs up to rounding); otherwise, or
 * with ISDF_W_PLAIN, they use U^q.  The FP64 path always uses U^q.
 *   n_frag    number of fragments (>= 1).
 *   n_f       [n_frag] orbitals per fragment (>= 1), host memory.
 *   C         [n_frag] pointers, fragment f: c128 [N_k][n_orb][n_f[f]].
 *   eri       [n_frag] pointers, fragment f: c128 [n_f]^4 output.
 *   flags     ISDF_FRAG_DEVICE if C[f] / eri[f] are device pointers;
 *             ISDF_FRAG_BLOCKS(n) to force n pair blocks per fragment.
 * Memory: the batch runs in sub-batches of consecutive fragments whose
 * workspace fits the free device memory; a fragment that does not fit alone
 * runs with its pairs (pq) in blocks (eqs. (19)-(20) over pair blocks: R^q of
 * a row block and of a column block and U^q of the row block are held at a
 * time, and the Hermitian contraction runs over block pairs), up to 32
 * blocks.  Results do not depend on the blocking (each output element is
 * summed in the same order).
 * Synchronous.  Error: ISDF_E_STATE before isdf_coulomb_kernel,
 * ISDF_E_NOMEM if a fragment does not fit even in 32 pair blocks.
 */
isdf_status isdf_fragment_eri(isdf_ctx ctx, isdf_precision prec, int32_t n_frag,
                              const int32_t* n_f, const void* const* C, void* const* eri,
                              uint32_t flags);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * fragment ERIs as isdf_fragment_eri (same kernels, bit-identical results),
 * with the whole workspace -- coefficient gather, psi, R^q, U^q, the FP64
 * contraction and the launch descriptors -- in a static device array of
 * ISDF_STATIC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends (4 MiB of it for descriptors).  The call allocates
 * and frees no device memory.  C[f] and eri[f] must be device pointers
 * (flags must include ISDF_FRAG_DEVICE).  Fragments run in sub-batches and
 * (pq) blocks that fit the array; a fragment that does not fit even in 32
 * pair blocks is refused with ISDF_E_NOMEM before any launch.  No part of
 * the array needs to start at zero.  Every call on a GPU shares that GPU's
 * array (also across contexts): calls that overlap in time on one GPU race
 * and must be serialised by the caller.  Synchronous.  Errors as
 * isdf_fragment_eri, ISDF_E_INVALID for host pointers.
 */
#define ISDF_STATIC_SCRATCH_BYTES (256ull << 20)
isdf_status isdf_fragment_eri_static(isdf_ctx ctx, isdf_precision prec, int32_t n_frag, const int32_t* n_f,
                                     const void* const* C, void* const* eri, uint32_t flags);

/*
 * A fragment batch captured as a HIP graph (the batched persistent launch of
 * Algorithm 2 replayed without host-side launch work, for callers that run the
 * same batch shape repeatedly).  isdf_graph_create runs the batch once on a
 * private stream and workspace (sizing every buffer, checking the result
 * paths), then captures the same launches and instantiates them.  Only device
 * pointers: C[f] and eri[f] as in isdf_fragment_eri with ISDF_FRAG_DEVICE.
 * Every replay reads C[f], X^k and W^q as they are at that time and writes
 * eri[f]: coefficients may be updated in place between replays, and a new
 * isdf_coulomb_kernel is seen by the next replay.  isdf_graph_launch replays
 * the graph after the work already queued on the context's stream and waits
 * for it.  Error: ISDF_E_STATE when no Coulomb kernel is current (create and
 * launch), ISDF_E_INVALID for bad arguments or host pointers.  The graph owns
 * its workspace until isdf_graph_destroy, which must come before the
 * context's isdf_destroy.
 */
typedef struct isdf_graph_s* isdf_graph;
isdf_status isdf_graph_create(isdf_ctx ctx, isdf_precision prec, int32_t n_frag, const int32_t* n_f,
                              const void* const* C, void* const* eri, isdf_graph* out);
isdf_status isdf_graph_launch(isdf_graph g);
isdf_status isdf_graph_destroy(isdf_graph g);

/*
 * Launch tiling of the fragment contraction, measured on the caller's batch.
 * Two runtime choices shape the GEMM launches of Algorithm 2: the number of
 * classes {q, -q} whose K ranges one ERI launch covers (the FP32 partial sums
 * then go into the FP64 accumulation once per launch) and the workgroups per
 * CU of the persistent tile loops.  isdf_autotune runs the batch (device
 * pointers, as isdf_graph_create) under each candidate -- the N_h classes in
 * one, two or three launches and the initial tiling, times {1, 2, 4, 8}
 * workgroups per CU --, twice each after a
 * warm-up, keeps the fastest for this context and, when `report` is not
 * NULL, fills it.  One workgroup per CU selects the ring pipeline of the
 * mixed-precision contraction (four LDS stages, the next stage's fragments
 * read during the current stage's MFMAs, one barrier a stage); its results
 * equal those of the two-stage pipeline bit for bit.  U^q keeps its own
 * pipeline whatever the tiling: two-stage with two workgroups a CU in
 * bf16x3, the ring in single bf16.  The eri[f]
 * hold the last candidate's results afterwards.  isdf_set_tiling sets the two
 * values directly (wg_per_cu 0 = 8 per CU).  A context starts at the most
 * classes a launch, at most 12, whose K range of one operand row in the
 * 8-byte mixed formats stays within 72 KB (12 up to N_IP = 768, 11 at
 * 800, 8 at 1040; balanced groups), and 2 workgroups per CU; at 12 classes that
 * is the tuner's choice on a 4x4x4 mesh with 64 fragments of 12-40
 * orbitals.  isdf_stats reports the current and the initial classes per
 * launch (eri_qgroup, eri_qgroup_initial) and wg_per_cu.  Results of every
 * tiling
 * meet the same error bounds; the FP32 partial sums change with the classes
 * per launch, so mixed results are bitwise reproducible for a fixed tiling
 * only.  Error: ISDF_E_STATE without a Coulomb kernel, ISDF_E_BUSY while
 * served requests are queued or running, ISDF_E_INVALID for bad arguments.
 */
typedef struct {
  int32_t eri_qgroup;   /* classes per ERI launch chosen */
  int32_t wg_per_cu;    /* workgroups per CU chosen */
  double ms;            /* batch time with the chosen tiling (best of two) */
  double ms_default;    /* batch time with the context's initial tiling (2 per CU) */
  int32_t n_tried;      /* candidates timed */
} isdf_tune_report;
isdf_status isdf_autotune(isdf_ctx ctx, isdf_precision prec, int32_t n_frag, const int32_t* n_f,
                          const void* const* C, void* const* eri, isdf_tune_report* report);
isdf_status isdf_set_tiling(isdf_ctx ctx, int32_t eri_qgroup, int32_t wg_per_cu);

/*
 * Served requests (continuous batching).  isdf_serve_start launches the
 * serving thread; isdf_submit queues one fragment (non-blocking) and returns
 * a ticket; the thread admits queued requests into batches while their HBM
 * footprint fits the budget and up to `max_inflight` batches are on the GPU,
 * so requests that arrive while others run join the next batch.  C and eri
 * are caller-owned and must stay valid until poll reports DONE, FAILED or
 * CANCELLED.  latency = submit -> completion observed (host monotonic clock).
 * isdf_fit and isdf_coulomb_kernel may run while serving only when no request
 * is queued or running (ISDF_E_BUSY otherwise); a request admitted while no
 * W^q exists ends FAILED.
 */
typedef struct {
  int32_t n_f;
  const void* C;        /* c128 [N_k][n_orb][n_f] */
  void* eri;            /* c128 [n_f]^4           */
  int32_t prec;         /* isdf_precision         */
  uint32_t flags;       /* ISDF_FRAG_DEVICE       */
  int32_t priority;     /* admission order: higher first, submission order
                           among equal priorities (0 = default)           */
} isdf_request;

isdf_status isdf_serve_start(isdf_ctx ctx, int32_t max_inflight, int32_t max_batch,
                             int64_t budget_bytes);
isdf_status isdf_submit(isdf_ctx ctx, const isdf_request* req, uint64_t* ticket);
/* Submit n requests at one instant (same submit time; admitted together when
 * they fit one batch).  tickets: [n] output.  All-or-nothing validation. */
isdf_status isdf_submit_n(isdf_ctx ctx, int32_t n, const isdf_request* reqs, uint64_t* tickets);
isdf_status isdf_poll(isdf_ctx ctx, uint64_t ticket, int32_t* state, double* latency_s);
isdf_status isdf_cancel(isdf_ctx ctx, uint64_t ticket);
/* Stops accepting requests, waits for everything queued, joins the thread. */
isdf_status isdf_serve_stop(isdf_ctx ctx);

/* JSON summary: sizes, ranks of Pi^q, per-stage device milliseconds of the
 * last call of each stage, served request counts.  Truncated to cap bytes. */
isdf_status isdf_stats(isdf_ctx ctx, char* json, int64_t cap);

/* Device milliseconds of a stage over the last call that ran it, measured
 * with HIP events on the stream the stage ran on ("metric_t", "metric_kconv",
 * "rhs", "chol", "grid_fft", "v_gemm", "w_solve", "frag_t", "frag_pair",
 * "frag_u", "frag_eri"); -1 if unknown. */
double isdf_stage_ms(isdf_ctx ctx, const char* name);
/* Sum of the device milliseconds and the number of intervals of a stage since
 * the context was created or isdf_stage_reset (served batches included). */
isdf_status isdf_stage_total(isdf_ctx ctx, const char* name, double* ms, int64_t* count);
isdf_status isdf_stage_reset(isdf_ctx ctx);

/* Memory planner: device bytes that isdf_create/fit/coulomb_kernel would hold
 * for these sizes with eta of every class resident (no allocation; q
 * batches need less), and the storage model of the paper's section on
 * diamond, N_k N_IP^2 + N_k N_IP N_AO complex128 elements. */
int64_t isdf_plan_bytes(const int32_t grid[3], const int32_t kmesh[3], int32_t n_orb,
                        int32_t n_ip);
int64_t isdf_storage_model_bytes(int64_t n_k, int64_t n_ip, int64_t n_ao);

/*
 * Checkpoint and resume of the fitted cell: the W^q of the paper's storage
 * model (section on the diamond cell at N_k = 1000) together with what the
 * fragment ERIs need besides it.  isdf_save writes, after isdf_coulomb_kernel,
 * a little-endian file: a 144-byte header
 *   char magic[8] = "ISDFCKP1"; uint32 version = 1; uint32 header_bytes = 144;
 *   int32 grid[3], kmesh[3], n_orb, n_ip, nh; uint32 flags;
 *   float64 lattice[9]; uint64 payload_bytes; uint64 checksum
 * then the payload
 *   int32 ip_index[n_ip]; int32 rank[nh] (rank of each Pi^q factor);
 *   c128 X[N_k][n_orb][n_ip]; c128 Pi[nh][n_ip][n_ip]; c128 W[nh][n_ip][n_ip]
 * where nh is the number of classes {q, -q} and class h holds the h-th q (C
 * order over the mesh) whose -q is not smaller; checksum = FNV-1a 64 of the
 * payload bytes.  isdf_load reads and checks the whole file on the host
 * (magic, version, sizes against the k mesh, length, checksum, ranks,
 * interpolation points) before any device call, then creates a context on
 * `hip_stream` whose fragment ERIs, served requests, graphs and test hooks
 * (isdf_get_metric, isdf_get_kernel, isdf_get_ivs) equal those of the saved
 * context bit for bit.  The restored context holds no orbitals: isdf_fit on it
 * is ISDF_E_STATE.  Errors: isdf_save ISDF_E_STATE before isdf_coulomb_kernel,
 * ISDF_E_INVALID when the file cannot be written; isdf_load ISDF_E_INVALID
 * for a missing, truncated, corrupted or inconsistent file (*out NULL, message
 * from isdf_last_error(NULL)), ISDF_E_NOMEM / ISDF_E_DEVICE as isdf_create.
 */
isdf_status isdf_save(isdf_ctx ctx, const char* path);
isdf_status isdf_load(isdf_ctx* out, const char* path, void* hip_stream);

/*
 * k-point Hartree-Fock Coulomb and exchange matrices from the resident W^q
 * (eq. (10) and the q = 0 term of eq. (9)), for density matrices P^k:
 *   rho^k_{IJ} = sum_{la sg} X^k_{I la} P^k_{la sg} conj(X^k_{J sg})
 *   K^k_{mu nu} = N_k^-1 sum_IJ conj(X^k_{I mu}) X^k_{J nu} sum_q W^q_{IJ} rho^{k+q}_{IJ}
 *   J^k_{mu nu} = N_k^-1 sum_I conj(X^k_{I mu}) X^k_{I nu} sum_J W^0_{IJ} n_J,
 *                 n_J = sum_k rho^k_{JJ}
 * i.e. J_{mu nu} = sum (mu nu|sg la) P_{la sg} and K_{mu nu} = sum
 * (mu la|sg nu) P_{la sg} over the supercell orbitals N_k^{-1/2} phi^k, for
 * the density matrix gamma(x, y) = N_k^-1 sum_k phi^k(x) P^k phi^k(y)^H.  K
 * is returned without the minus sign with which eq. (10) enters the Fock
 * matrix; q is counted as in W^q of this library.  The q sum is a
 * convolution over the k mesh, done in place on rho (FP64 k transforms in
 * LDS); the other steps are FP64 MFMA products.  FP64 throughout.
 *   dm     c128 [N_k][n_orb][n_orb], row mu column nu.
 *   j_out, k_out  c128 [N_k][n_orb][n_orb], either may be NULL (not computed).
 *   flags  ISDF_HF_DEVICE: dm, j_out, k_out are device pointers (else host).
 * Device workspace N_k N_IP^2 + N_k n_orb N_IP complex numbers (17.3 + 0.9 GB
 * at N_k = 1000, N_IP = 1040), freed on return; the idle workspace of
 * isdf_fragment_eri is handed back first when the device is full.
 * Synchronous.  Errors: ISDF_E_STATE before isdf_coulomb_kernel,
 * ISDF_E_INVALID for null or (with ISDF_HF_DEVICE) non-device pointers and
 * for K on meshes of more than 2048 k points, ISDF_E_NOMEM, ISDF_E_DEVICE.
 */
#define ISDF_HF_DEVICE 0x1u
isdf_status isdf_hf_jk(isdf_ctx ctx, const void* dm, void* j_out, void* k_out, uint32_t flags);

/*
 * k-point opposite-spin MP2 energy in the imaginary-time form (eqs. (11)-(15))
 * from the resident W^q, per unit cell in Hartree (E_SOS-MP2 = 1.3 E_OS, eq.
 * (11)).  Canonical orbitals psi^k_p = sum_mu C^k_{mu p} phi^k_mu with
 * energies e^k_p, the first n_occ of every k occupied; Y^k = X^k C^k; m the
 * midpoint between the highest occupied and the lowest virtual energy:
 *   Go^k(tau) = Y_o e^{+tau (e_i - m)} Y_o^H,  Gv^k(tau) = Y_v e^{-tau (e_a - m)} Y_v^H
 *   chi^q  = N_k^-1 sum_k Gv^k o conj(Go^{k+q}),  chit^q = N_k^-1 sum_k Go^k o conj(Gv^{k+q})
 *   F(tau) = N_k^-1 sum_q tr[W^q chi^q W^q chit^q],   E_OS = -sum_n weight_n F(tau_n)
 * (the Green's functions are the decaying ones; q as in W^q of this
 * library; E_OS < 0).  Per tau: the Green's functions as Hermitian FP64 MFMA
 * products, chi and chit of one q per class {q, -q} by one in-place
 * convolution over the k mesh (LDS), W chi and chit W as FP64 MFMA products,
 * the trace as an element-wise dot; a class with q != -q counts twice (its
 * -q term is the conjugate).  FP64 throughout.
 *   mo_coeff    c128 [N_k][n_orb][n_mo] (ISDF_MP2_DEVICE: device, else host).
 *   mo_energy   float64 [N_k][n_mo], host; occupied below virtual.
 *   tau, weight float64 [n_tau], host: a quadrature of [0, inf) (caller's).
 *   integrand_out  float64 [n_tau] or NULL: F(tau_n).
 *   class_out   float64 [n_tau][nh] or NULL: the contribution of class h to
 *               F(tau_n) (class h = the h-th q of the mesh in C order whose -q
 *               is not smaller).
 *   e_os_out    float64: E_OS.
 * Device workspace 2 N_k N_IP^2 + nh N_IP^2 complex numbers plus
 * N_k N_IP n_mo x 2 (34.6 + 8.7 + 1.7 GB at N_k = 1000, N_IP = 1040),
 * freed on return.  Synchronous.  Errors: ISDF_E_STATE before
 * isdf_coulomb_kernel; ISDF_E_INVALID for null pointers, bad counts, energies
 * without a gap, negative or non-finite tau, more than 2048 k points;
 * ISDF_E_NOMEM, ISDF_E_DEVICE.
 */
#define ISDF_MP2_DEVICE 0x1u
isdf_status isdf_sos_mp2(isdf_ctx ctx, const void* mo_coeff, const double* mo_energy, int32_t n_mo,
                         int32_t n_occ, int32_t n_tau, const double* tau, const double* weight,
                         double* integrand_out, double* class_out, double* e_os_out, uint32_t flags);

/*
 * k-point direct RPA correlation energy (eq. (16)) from the resident W^q,
 * per unit cell in Hartree, with the polarisabilities of isdf_sos_mp2:
 *   chi^q(iw_m) = -sum_n [gamma_mn chi^q(tau_n) + conj(gamma_mn) chit^q(tau_n)],
 *             the time integral of both orderings with the caller's transform
 *             gamma_mn, which maps exp(-D tau_n) to 1/(D - i w_m) for the
 *             excitation energies D of the system: a plain quadrature
 *             (gamma_mn = weight_n exp(i w_m tau_n), accurate only where the
 *             time grid resolves exp(i w tau)) or a least-squares fit over the
 *             range of D (accurate at every frequency),
 *   E_dRPA    = sum_m omega_weight_m F(w_m),
 *   F(w)      = (pi N_k)^-1 sum_q Re[ln det(1 - chi^q(iw) W^q) + tr(chi^q(iw) W^q)]
 * (the integral over w in (-inf, inf) of eq. (16) folded onto [0, inf):
 * chi^q(-iw) = chi^q(iw)^H), and its second-order term
 * (pi N_k)^-1 sum_q -1/2 Re tr[(chi W)^2], which is the opposite-spin MP2
 * energy.  chi^q(iw) is not Hermitian without time-reversal symmetry, so
 * Re ln det(1 - P) is taken as 1/2 ln det(A^H A), A = 1 - P, from a blocked
 * FP64 Cholesky factor; P, A^H A and the time convolutions are FP64 (MFMA for
 * the products).  One q per class {q, -q} (the -q term is the conjugate).
 * The frequencies are processed in batches that fit the device memory (the
 * time loop runs once per batch).
 *   mo_coeff, mo_energy, n_mo, n_occ  as isdf_sos_mp2 (ISDF_DRPA_DEVICE:
 *               mo_coeff in device memory).
 *   tau        float64 [n_tau], host: the times of the polarisabilities.
 *   omega_weight  float64 [n_omega], host: weights of a quadrature of [0, inf)
 *               in frequency.
 *   transform  c128 [n_omega][n_tau], host: gamma_mn.
 *   integrand_out  float64 [n_omega] or NULL: F(w_m).
 *   class_out   float64 [n_omega][nh] or NULL: the contribution of class h to
 *               F(w_m) (class order as isdf_sos_mp2).
 *   e_drpa_out  float64: E_dRPA;  e_second_out  float64 or NULL: the
 *               second-order term on the same grids.
 * Device workspace as isdf_sos_mp2 plus 3 nh N_IP^2 and, per frequency of a
 * batch, nh N_IP^2 complex numbers; freed on return.  Synchronous.  Errors:
 * as isdf_sos_mp2 (non-finite transform or weights: ISDF_E_INVALID);
 * ISDF_E_NUMERIC when 1 - chi W is singular; ISDF_E_NOMEM when not even one
 * frequency fits.
 */
#define ISDF_DRPA_DEVICE 0x1u
isdf_status isdf_drpa(isdf_ctx ctx, const void* mo_coeff, const double* mo_energy, int32_t n_mo, int32_t n_occ,
                      int32_t n_tau, const double* tau, int32_t n_omega, const double* omega_weight,
                      const void* transform, double* integrand_out, double* class_out, double* e_drpa_out,
                      double* e_second_out, uint32_t flags);

isdf_status isdf_destroy(isdf_ctx ctx);
/* Message of the last failed call on ctx; with ctx == NULL, the message of the
 * last failed isdf_create or isdf_load on the calling thread ("null context"
 * if none). */
const char* isdf_last_error(isdf_ctx ctx);
const char* isdf_version(void);

#ifdef __cplusplus
}
#endif
#endif /* ISDF_H */
