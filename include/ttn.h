/*
 * ttn.h - C ABI of the MI355X (gfx950) binary tree tensor network sweep.
 *
 * The library runs the energy-minimisation sweep of a uniform binary tree
 * tensor network (TTN) for a periodic effective chain
 *     H = sum_j [ h1_j + sum_k A_{k,j} B_{k,j+1} ],
 * following Milsted, Ganahl, Leichenauer, Hidary, Vidal, "TensorNetwork on
 * TensorFlow: A Spin Chain Application Using Tree Tensor Networks"
 * (arXiv:1905.01331): the ansatz of Sec. II.C (isometries w of
 * Eq. (constraint), one per layer by translation invariance, Sec. III; top
 * tensor v of Eq. (normalization)), the environment of Sec. III.A
 * (Figs. 2(b), 3, 4(b)), the SVD/polar update of Sec. III.B (Fig. 4(c-d),
 * Fig. 10(a)) and the sweep of Secs. IV-V.
 *
 * Levels tau = 0..n-1 (L = 2^n effective sites, level tau has L/2^tau
 * sites, level n-1 has 2).  Bond dimensions chi_0 = d,
 * chi_tau = min(chi_{tau-1}^2, chi).  Layer tau = 1..n-1 holds one isometry
 * w_tau[a; l, r] of shape (chi_tau, chi_{tau-1}, chi_{tau-1}), row-major with
 * r fastest, rows orthonormal.  The top tensor v is chi_{n-1} x chi_{n-1},
 * row-major, unit Frobenius norm.  All matrices are real, row-major, ket
 * index first.
 *
 * Memory and streams.  The caller allocates ONE device workspace of at least
 * ttn_workspace_bytes() bytes and passes it to ttn_init(); the library never
 * allocates device memory itself and lays out all tensors inside it.  Host
 * arrays passed in are copied before the call returns.  Every stage call is
 * enqueued asynchronously on the caller's HIP stream (hipStream_t passed as
 * void*); ttn_energy, ttn_get_tensor, ttn_get_operator and ttn_stats
 * synchronise that stream.
 *
 * Errors.  Every call returns a ttn_status: 0 = success, < 0 = error (the
 * handle is left unchanged and ttn_last_error() describes it), > 0 = a
 * warning (the call completed).  No exception crosses the ABI.  A handle is
 * not thread-safe; distinct handles on distinct streams are independent.
 */
#ifndef TTN_H
#define TTN_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ttn_ctx* ttn_handle;
typedef int ttn_status;

enum {
  TTN_OK = 0,
  TTN_WRANK = 1,        /* an environment was numerically rank deficient
                           (sigma_min/sigma_max < 1e-14): the polar factor is
                           not unique there and was completed
                           deterministically; or (ttn_energy, evd_update = 1)
                           an isometry is orthonormal only to the precision
                           of the squared environment                         */
  TTN_WNOCONV = 2,      /* the top eigensolver stopped at its iteration budget
                           above its residual target                          */
  TTN_WPROF = 3,        /* ttn_profile_read: launches were not timed (event
                           pool full); the returned record is incomplete       */
  TTN_EINVAL = -1,      /* invalid argument or configuration                  */
  TTN_ENOMEM = -2,      /* workspace smaller than ttn_workspace_bytes()        */
  TTN_EHIP = -3,        /* a HIP runtime call failed                          */
  TTN_ENONFINITE = -4,  /* NaN or Inf in a host input                         */
  TTN_ENOCONV = -5,     /* a Jacobi eigensolver stopped at its sweep limit     */
  TTN_EORTHO = -6,      /* an updated isometry failed the orthonormality check */
  TTN_ESTATE = -7       /* stage called out of the order of the sweep         */
};

/* Arithmetic of the bulk contractions (ascend, descend, environment).  The
 * polar update, the orthonormality check, the top eigensolver and the
 * energy always run in float64. */
enum {
  TTN_FP64 = 0,        /* float64 everywhere                                  */
  TTN_FP32 = 1,        /* float32 operands, float32 MFMA accumulation          */
  TTN_SPLIT_BF16 = 2   /* each float32 operand x = hi + lo with bf16 hi, lo;
                          hi*hi + hi*lo + lo*hi on bf16 MFMA, float32 accumulate */
};

enum { TTN_DESCEND_RHO = 0, TTN_DESCEND_DRESSED = 1 };
#define TTN_TOP (-1)

/* Kinds for ttn_get_operator (level-tau one-site matrices, chi_tau^2). */
enum {
  TTN_OP_H = 0,     /* one-site term h^(tau), shift included (level 0: h1 - c I) */
  TTN_OP_A = 1,     /* product term A_k^(tau)                                  */
  TTN_OP_B = 2,     /* product term B_k^(tau)                                  */
  TTN_OP_RHO = 3,   /* position-averaged one-site RDM rho^(tau) (descend cache) */
  TTN_OP_RBAR = 4,  /* A_k-dressed two-site RDM seen from the B site, level tau  */
  TTN_OP_LBAR = 5,  /* B_k-dressed two-site RDM seen from the A site, level tau  */
  TTN_OP_ENV = 6    /* environment of w_tau (chi_tau x chi_{tau-1}^2), last ttn_env */
};

typedef struct ttn_config {
  int L;              /* effective sites: power of two, >= 4                  */
  int d;              /* effective site dimension (2, or 2^L_y for a torus)   */
  int chi;            /* bond-dimension cap, >= 1                             */
  int D;              /* number of product terms, >= 0                        */
  const double* h1;   /* host, d*d, symmetric one-site term                   */
  const double* A;    /* host, D*d*d: A_k acts on site j                      */
  const double* B;    /* host, D*d*d: B_k acts on site j+1; each pair (A_k,B_k)
                         is both symmetric or both antisymmetric              */
  double shift;       /* c with every bond term minus c negative semidefinite;
                         NaN selects the largest eigenvalue of the bond term
                         1/2(h1 x I + I x h1) + sum_k A_k x B_k              */
  int ly;             /* physical spins per effective site (energy per spin
                         divides by L*ly), >= 1                               */
  int precision;      /* TTN_FP64, TTN_FP32 or TTN_SPLIT_BF16                 */
  unsigned long long seed; /* isometries when w0 == NULL: Gaussian entries
                         from a counter-based generator (SplitMix64 +
                         Box-Muller) made orthonormal by the polar update     */
  const double* const* w0; /* optional host array of n-1 pointers, layer tau
                         at w0[tau-1] with shape (chi_tau, chi_{tau-1}^2)     */
  const double* v0;   /* optional host chi_{n-1}^2 start vector of the top
                         eigensolver (else a fixed deterministic vector)      */
  int krylov;         /* Lanczos basis size per restart (0: 24)               */
  int restarts;       /* Lanczos restarts per top update (0: 8)               */
  double lanczos_tol; /* target ||H v - lambda v|| / max(1, |lambda|) (0: 1e-12) */
  int keep_gauge;     /* 0 (default): after each update the output index of
                         w_tau is rotated into the singular basis of its
                         environment and the layer above (or v) absorbs the
                         inverse rotation, which leaves the state unchanged
                         and keeps the next environment's Gram matrix nearly
                         diagonal; 1: store -polar(Env) as is              */
  int evd_update;     /* 0 (default): the polar factor to working accuracy
                         (Gram refreshes until the rows are orthogonal);
                         1: the eigenvalue-decomposition variant of the
                         appendix (Fig. 10(b)): one Gram matrix Env Env^T =
                         U S^2 U^T and w = -U S^-1 U^T Env, cheaper but with
                         the precision of the squared environment (relative
                         errors of order eps (s_max / s_min)^2)              */
} ttn_config;

/* Bytes of device workspace needed by ttn_init for these configs. */
ttn_status ttn_workspace_bytes(const ttn_config* cfgs, int batch, size_t* bytes);

/* Validates the configs, lays out the caller-owned device workspace
 * (`workspace`, `bytes`, 256-byte aligned), copies the host inputs, builds
 * or loads the isometries, ascends every level, solves the top tensor and
 * computes the energy (Sec. III; initial state of the sweep).  `stream` is a
 * hipStream_t (NULL = default stream).  On success *out owns no device memory;
 * the workspace must outlive the handle. */
ttn_status ttn_init(const ttn_config* cfgs, int batch, void* workspace, size_t bytes,
                    void* stream, ttn_handle* out);

/* Ascends the one-site term and the product terms through layers
 * tau_from..tau_to (1 <= tau_from <= tau_to <= n-1), Fig. 3 / Fig. 4(b):
 *   h' = w S w^T,  A'_k = w (I x A_k) w^T,  B'_k = w (B_k x I) w^T
 * with S = h x I + I x h + sum_k A_k x B_k applied to the legs of w. */
ttn_status ttn_ascend(ttn_handle h, int tau_from, int tau_to);

/* what = TTN_DESCEND_RHO: position-averaged one-site RDMs rho^(tau) for
 *   tau = n-1..1 from v (cache for the whole sweep; `tau` is ignored).
 * what = TTN_DESCEND_DRESSED: the two-site information Rbar_k^(tau),
 *   Lbar_k^(tau) for the update of layer tau (1 <= tau <= n-1): A_k, B_k of
 *   level tau-1 are carried up to the top with the current layers, dressed by
 *   v and descended back to level tau (Sec. III.A, Fig. 3). */
ttn_status ttn_descend(ttn_handle h, int tau, int what);

/* Environment of w_tau (Sec. III.A), same index shape as w_tau:
 *   Env = rho o (S w) + sum_k Rbar_k o (B_k .l w) + sum_k Lbar_k o (A_k .r w).
 * Requires ttn_descend(tau, DRESSED) since the last change of layer tau. */
ttn_status ttn_env(ttn_handle h, int tau);

/* tau in 1..n-1: w_tau <- -polar(Env) = -U V^T for the thin SVD
 *   Env = U S V^T (Sec. III.B, Fig. 10(a)), in float64, followed by the check
 *   ||W W^T - I||_F <= max(1e-10, 64 eps a^(3/2)), a the largest bond
 *   dimension (reported as TTN_EORTHO by ttn_energy).  Unless
 *   keep_gauge is set the stored tensor is U^T w_tau = -V^T and w_{tau+1}
 *   (or v when tau = n-1) absorbs U on its input legs (same state).  Does not
 *   re-ascend.
 * tau == TTN_TOP: v <- lowest eigenvector of the top Hamiltonian (Lanczos,
 *   float64, warm-started from the current v) and the energy. */
ttn_status ttn_update(ttn_handle h, int tau);

/* Synchronises the stream and writes the energy per physical spin
 * (E + c L) / (L ly) of each batch member to e_per_site[batch] (host): the
 * energy per site of Sec. IV, E the lowest eigenvalue of the shifted top
 * Hamiltonian and L ly the number of spins (a torus column of ly spins is
 * one site).  Errors: TTN_EHIP when a Jacobi solve aborted, TTN_EORTHO when
 * an updated isometry failed its orthonormality check, TTN_ENOCONV when a
 * Jacobi solve of the last sweep stopped at its sweep limit without
 * converging; warnings: TTN_WRANK (see evd_update), TTN_WNOCONV when the
 * last top update stopped at its restart budget above its residual target. */
ttn_status ttn_energy(ttn_handle h, double* e_per_site);

/* nsweeps full sweeps (Secs. IV-V): descend(RHO); for tau = 1..n-1 {
 * descend(tau, DRESSED); env(tau); update(tau); ascend(tau, tau) };
 * update(TOP).  The members of a batch run their layer steps side by side on
 * internal streams forked from and joined back into the handle's stream.
 * use_graph = 0: eager launches; update(TOP) reads its convergence on the
 * host after every restart and stops launching once every member converged
 * (TTN_WNOCONV when the restart budget ran out first).
 * use_graph != 0: the layer part is captured into a HIP graph on the first
 * such call and replayed on every later one; it holds no host
 * synchronisation (the polar update's optional extra refresh is decided on
 * the device).  The top update is replayed from a second graph that holds a
 * planned number of Lanczos restarts: a flag set on the device when the
 * residual meets its target makes the kernels of the later restarts return
 * at once.  use_graph = 2: the plan is the whole restart budget, and nothing
 * is read back (ttn_energy reports a top update that did not converge).
 * use_graph = 1: the plan is the number of restarts the slowest member has
 * needed so far (one graph per plan, kept); one host read after the replay
 * runs the rest of the budget eagerly for a member that needs more, and
 * raises the plan.  The graphs refer to the handle's workspace only, so
 * ttn_set_tensor between sweeps is honoured.  Ignored while profiling is on.
 * Results are identical in every mode. */
ttn_status ttn_sweep(ttn_handle h, int nsweeps, int use_graph);

/* nsweeps grouped sweeps: a schedule of our own beside the paper's (the
 * update of Sec. III.B, the sweep of Sec. IV).  The layers are split into
 * groups (groups = 1: every layer; groups = 2: the odd layers, then the even
 * ones); every layer of a group takes its environment from the same state.
 * With nothing changed in between, the operators that a layer's dressed chain
 * carries up are the ascended operators themselves, so one top-down pass
 * yields the two-site information of every level: per group, descend(RHO),
 * one pass of the chains with env and update of the group's layers on the
 * way down, then every layer is ascended again; after the last group,
 * update(TOP).  The dressed chains take one pass per group, against one
 * chain per layer in ttn_sweep.  groups = 1 updates neighbouring
 * layers from the same state and may raise the energy of strongly coupled
 * models; groups = 2 keeps neighbours apart.  Batches run their launch groups
 * one after another on the handle's stream.  use_graph != 0: the layer part
 * is captured into a HIP graph (one per grouping) on the first such call and
 * replayed, and update(TOP) as in ttn_sweep; results are identical in every
 * mode.
 * TTN_EINVAL for groups outside {1, 2}; TTN_ESTATE when a level's operators
 * are stale; otherwise as ttn_sweep. */
ttn_status ttn_sweep_grouped(ttn_handle h, int nsweeps, int groups, int use_graph);

/* Checkpoint / parity access to the float64 master tensors of member b:
 * tau in 1..n-1 selects w_tau (chi_tau*chi_{tau-1}^2 doubles), tau == TTN_TOP
 * selects v (chi_{n-1}^2 doubles).  set_tensor invalidates every cached
 * operator above the layer; call ttn_ascend before the next stage. */
ttn_status ttn_get_tensor(ttn_handle h, int b, int tau, double* host);
ttn_status ttn_set_tensor(ttn_handle h, int b, int tau, const double* host);

/* Copies a level-tau one-site matrix (kind TTN_OP_*, product term k) of
 * member b to host float64 (chi_tau^2 doubles; TTN_OP_ENV: the last
 * environment of layer tau, chi_tau*chi_{tau-1}^2 doubles). */
ttn_status ttn_get_operator(ttn_handle h, int b, int level, int kind, int k, double* host);

typedef struct ttn_stats_t {
  double energy;          /* energy per physical spin after the last update    */
  double lambda;          /* lowest eigenvalue of the shifted top Hamiltonian */
  double lanczos_resid;   /* ||H v - lambda v|| of the last top update        */
  double ortho_err_max;   /* max ||W W^T - I||_F of the updates since init    */
  double sigma_ratio_min; /* min sigma_min/sigma_max of the environments       */
  double shift;           /* c                                                 */
  double flops_bulk;      /* algorithmic bulk flops of one sweep              */
  double flops_fp64;      /* algorithmic float64 flops of one sweep           */
  int n_levels;           /* n                                                 */
  int lanczos_iters;      /* Krylov steps of the last top update (restarts
                             that ran x the Krylov space)                     */
  int jacobi_sweeps[4];   /* Jacobi sweeps of the last polar update's three
                             refreshes and of the last Lanczos projection     */
  double e_prev;          /* energy per physical spin before the last top
                             update (0 before the first one)                  */
  double bytes_hbm;       /* algorithmic bytes of the products of the last
                             sweep (each operand read once, each result
                             written once, in the precision it is stored in):
                             the layer part as last launched or captured, plus
                             the last top update                              */
} ttn_stats_t;

ttn_status ttn_stats(ttn_handle h, int b, ttn_stats_t* out);

/* Autotuning of the contraction launches, for the whole process (all
 * handles).  mode 0: default launch shapes (default); 1: the first time a
 * product of a new shape and layout is run eagerly (not under graph capture)
 * with beta = 0, its candidate launch shapes (float64 output tile 64 x 64,
 * 128 x 64 or 64 x 128; the order in which tiles are handed to the XCDs) are timed with
 * HIP events on the handle's stream (this synchronises that stream) and the
 * fastest is kept; 2: kept choices only.  Kept choices are used in every mode
 * but 0, also inside captured graphs.  mode -1 leaves the mode unchanged.
 * entries (host, may be NULL) receives the number of kept choices.  A choice
 * never changes a result: the split of a contraction into partial sums, and
 * the instruction sequence of every output element, depend on the product's
 * shape alone, so every mode gives the same bits. */
ttn_status ttn_autotune(int mode, int* entries);

/* The kept launch choices written to a text file (path, host string), and
 * read back (merged into the table; entries, may be NULL, receives the
 * number read).  TTN_EINVAL when the file cannot be written, read or parsed;
 * a failed load leaves the table unchanged. */
ttn_status ttn_autotune_save(const char* path);
ttn_status ttn_autotune_load(const char* path, int* entries);

/* Event timing of the contraction classes (apply_r, apply_l, close,
 * left_mul, close_l, close_r, top_mm, polar_gemm, jacobi, lanczos_gemm) and
 * of the product kernels one by one.
 * ttn_profile(h, 1) clears the record and brackets every later launch of a
 * class with hipEventRecord on the stream it runs on; ttn_profile(h, 0)
 * stops.  While it is on, every launch of a product kernel (by any handle of
 * the process; the last handle to turn profiling on receives them) is also
 * bracketed alone, without its split-K reduction, under the kernel's
 * instantiation name (e.g. "gemm_mfma_kernel<2, true, false>", the name a
 * kernel trace shows).  Graph sweeps are not timed (a profiled sweep runs
 * eagerly).  ttn_profile_read synchronises and returns one entry per class
 * and then per kernel, with its launch count, summed elapsed milliseconds and
 * algorithmic flops (2 M N K per product) and bytes (operands read once,
 * result written once, in the precision the kernel reads and writes).
 * Classes come first, in the order above. */
typedef struct ttn_profile_entry {
  char name[48];
  int launches;
  double ms;
  double flops;
  double bytes;
} ttn_profile_entry;
ttn_status ttn_profile(ttn_handle h, int enable);
ttn_status ttn_profile_read(ttn_handle h, ttn_profile_entry* out, int max_entries, int* n_out);

/* Entanglement of a block of sites (Sec. V, the entanglement spectrum and
 * entropy equations): the eigenvalues p_alpha of the reduced density matrix
 * on the upper bond index of an isometry of layer tau, i.e. of a block of
 * 2^tau effective sites (tau = 0: one site; tau = n-1: half of the chain),
 * and S = -sum_alpha p_alpha log2 p_alpha.  The entanglement spectrum is
 * lambda_alpha = -log2 p_alpha.
 *   which = TTN_ENT_AVERAGE: the density matrix averaged over the positions
 *     of layer tau (what the sweep descends; every block of a uniform tree
 *     hangs from the same map, so this is also the spectrum of the average
 *     of the blocks' density matrices);
 *   which = TTN_ENT_LEFTMOST: the block of the first 2^tau sites (at the top
 *     v v^T, then one level down the left child of the block above, the
 *     right child traced out).
 * Computed in float64 from the current isometries and top tensor of member
 * b (descents, then a Jacobi eigensolver and a sort on the device).
 * p (host, chi_tau doubles) receives the spectrum in descending order (tiny
 * negative values are rounding), entropy (host) S.  Synchronises the stream;
 * does not change the sweep's state. */
enum { TTN_ENT_AVERAGE = 0, TTN_ENT_LEFTMOST = 1 };
ttn_status ttn_entanglement(ttn_handle h, int b, int tau, int which, double* p, double* entropy);

/* The same for the block of node `node` of level tau, i.e. the 2^tau sites
 * node 2^tau .. (node+1) 2^tau - 1 (node in 0..(L >> tau) - 1; node 0 is
 * TTN_ENT_LEFTMOST).  Its matrix is descended along its own path: at level
 * n-1 v v^T for the left half, v^T v for the right half; one level down the
 * left child (C_L) or the right child (C_R) of the node above, as the bits of
 * `node` say.  TTN_EINVAL for a node or level outside the tree. */
ttn_status ttn_entanglement_node(ttn_handle h, int b, int tau, long long node, double* p, double* entropy);

/* Position-resolved reading of the state of member b (the same uniform tree,
 * its nodes read one by one instead of averaged over positions; the energy
 * as a sum of local terms, Eqs. (H1D) and (1)-(5), its two-site terms met at
 * the node where their sites first share a causal cone, Fig. 3).
 *
 * ttn_local_energies fills, on the host,
 *   site[j] = <h1_j>                          (j = 0..L-1)
 *   bond[j] = sum_k <A_{k,j} B_{k,j+1}>       (site L is site 0)
 * for the Hamiltonian as given (no shift), so sum(site) + sum(bond) is the
 * energy of the state (the per-site energy of ttn_energy times L * ly).  It
 * also leaves in `work` the reduced density matrix on the upper bond of every
 * node: level tau has L >> tau nodes, node m covering the sites
 * m 2^tau .. (m+1) 2^tau - 1 (tau = 0: site m), each a chi_tau x chi_tau
 * row-major float64 matrix, node m at byte offset
 * ttn_positions_offset(h, b, tau) + 8 m chi_tau^2.  Level n-1 holds v v^T
 * and v^T v; node 2m (2m+1) of level tau-1 is the left (right) child of
 * node m of level tau, the other child traced out.
 *
 * Computed in float64 from the master isometries and top tensor, whatever
 * the bulk precision.  The handle's state is not changed (no stage order
 * applies).  work: device memory of the caller, 256-byte aligned, at least
 * ttn_positions_bytes(h, b) bytes (the matrices of every level plus scratch
 * of two chi^3 slices); a larger buffer lets more parents share each launch
 * of the descent, up to 256 MB of intermediates per launch (at chi = 256 the
 * minimum already reaches that).  Synchronises the stream.
 * TTN_EINVAL for a bad handle, member or pointer, or an unaligned work;
 * TTN_ENOMEM when bytes is below the minimum; TTN_EHIP from the runtime. */
ttn_status ttn_positions_bytes(ttn_handle h, int b, size_t* bytes);
ttn_status ttn_positions_offset(ttn_handle h, int b, int tau, size_t* offset);
ttn_status ttn_local_energies(ttn_handle h, int b, void* work, size_t bytes, double* site, double* bond);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid allocation): ttn_local_energies
 * with its work buffer in a static device array of the library,
 * TTN_NOALLOC_SCRATCH_BYTES (64 MiB) per GPU, held until the process ends,
 * instead of memory the caller brings.  It calls no allocating routine.
 * Inputs (the handle's state) and outputs (site, bond on the host) as for
 * ttn_local_energies, with the same results as ttn_local_energies given a
 * work buffer of TTN_NOALLOC_SCRATCH_BYTES bytes.  TTN_ENOMEM when member b
 * needs more than the static scratch (ttn_positions_bytes above
 * TTN_NOALLOC_SCRATCH_BYTES; e.g. L = 1024 at chi = 64 fits, L = 4096 at
 * chi = 256 does not); TTN_EINVAL, TTN_EHIP as for ttn_local_energies.
 * Every call on one GPU uses that GPU's one array, which keeps the last
 * call's contents (the computation writes every entry it reads): calls that
 * overlap on one GPU (from several threads or streams) race and must not be
 * made.  Synchronises the stream. */
#define TTN_NOALLOC_SCRATCH_BYTES (64u << 20)
ttn_status ttn_local_energies_noalloc(ttn_handle h, int b, double* site, double* bond);

/* ------------------------------------------------------------------------
 * Position-resolved network: every node (tau, m) its own isometry
 * w^(tau, m) (Sec. II.C labels the isometries by layer and position; the
 * translation-invariant Hamiltonians of Sec. III let the paper take them
 * equal along a layer, which the functions above do).  Float64 throughout.
 * Node m of level tau covers sites m 2^tau .. (m + 1) 2^tau - 1; its input
 * legs are nodes 2m (left) and 2m + 1 (right) of level tau - 1.
 *
 * A sweep (Sec. IV with each layer split by parity): layers bottom-up; in a
 * layer first the even then the odd nodes, every node of a parity group
 * updated from one state (such nodes are never neighbours: each group is an
 * exact block step), w <- -polar(Env) (Sec. III.B) for each; then the top
 * tensor as the lowest eigenvector of the top Hamiltonian, whose two sites
 * now carry different operators (Lanczos, as for ttn_update(TTN_TOP)).
 * Energies and errors as for the uniform network; the energy is the top
 * eigenvalue plus c L, divided by L ly.
 * ------------------------------------------------------------------------ */
typedef struct ttn_pos_ctx* ttn_pos_handle;

typedef struct ttn_pos_config {
  int L, d, chi, D;   /* as ttn_config                                         */
  const double* h1;   /* host d*d; A, B: host D*d*d (as ttn_config)            */
  const double* A;
  const double* B;
  double shift;       /* NaN: the largest eigenvalue of the bond term          */
  int ly;             /* spins per effective site                             */
  unsigned long long seed; /* start vector of the first top solve when v0 is
                         NULL (counter-based Gaussian, as ttn_config)         */
  const double* const* w0; /* required host array of n-1 pointers: w0[tau-1]
                         holds the L_tau isometries of layer tau, node-major,
                         each chi_tau x chi_{tau-1} x chi_{tau-1}
                         (L_tau = L >> tau)                                   */
  const double* v0;   /* optional host chi_{n-1}^2 start vector               */
  int krylov, restarts;  /* as in ttn_config, 0: 24, 8                         */
  double lanczos_tol;    /* as in ttn_config, 0: 1e-12                         */
  int chunk_nodes;    /* nodes per launch chunk at most (0: as many as 8 GiB of
                         staging holds); results do not depend on it beyond
                         rounding                                             */
} ttn_pos_config;

/* Workspace: the per-node arrays (isometries, operators, density matrices
 * and edge information of every node, the descent's cache: each about the
 * size of all isometries, so about five times the isometries' bytes), the
 * top solver's buffers, and staging of at most 8 GiB per launch chunk.
 * Same errors as ttn_workspace_bytes; TTN_EINVAL when w0 or one of its
 * layers is NULL. */
ttn_status ttn_pos_workspace_bytes(const ttn_pos_config* cfg, size_t* bytes);
/* Copies the inputs, ascends every node's operators and solves the top
 * problem (v0 or the seeded vector as the start).  Errors as ttn_init;
 * TTN_WNOCONV when the first top solve ended above its target. */
ttn_status ttn_pos_init(const ttn_pos_config* cfg, void* workspace, size_t bytes, void* stream,
                        ttn_pos_handle* out);
/* nsweeps sweeps (above).  TTN_EHIP / TTN_ENOCONV when a polar Jacobi solve
 * aborted / used its sweep limit; TTN_WNOCONV from the top solver. */
ttn_status ttn_pos_sweep(ttn_pos_handle h, int nsweeps);
/* e[0] = top eigenvalue lambda, e[1] = energy per spin of the current state. */
ttn_status ttn_pos_energy(ttn_pos_handle h, double* e);
/* rho, X, Y of every node of every level from the current tensors (read
 * back with ttn_pos_get(TTN_POS_DX)).  Synchronises the stream. */
ttn_status ttn_pos_descend(ttn_pos_handle h);
/* The environments of the nodes parity, parity + 2, .. of level tau (1 <=
 * tau < n) from the current tensors, into host (count x chi_tau x
 * chi_{tau-1}^2, count = L_tau / 2); the state is not changed. */
ttn_status ttn_pos_env(ttn_pos_handle h, int tau, int parity, double* host);
/* Copies a block to the host:
 *   TTN_POS_W   (level >= 1) the L_tau isometries, node-major;
 *   TTN_POS_OPS the operators [h, A_1..A_D, B_1..B_D] of each node (chi_tau^2
 *               each, node-major; level 0 one block: h1 - c I, A, B), h the
 *               sum of the terms inside the node's block, A_k its last site's
 *               and B_k its first site's edge operator;
 *   TTN_POS_DX  [rho, X_1..X_D, Y_1..Y_D] of each node as of the last
 *               ttn_pos_descend: X_k pairs with B_k (the bond arriving at the
 *               block's first site), Y_k with A_k (the bond leaving its last);
 *   TTN_POS_TOP the top tensor (level ignored). */
enum { TTN_POS_W = 0, TTN_POS_OPS = 1, TTN_POS_DX = 2, TTN_POS_TOP = 3 };
ttn_status ttn_pos_get(ttn_pos_handle h, int what, int level, double* host);
/* Counters of the last sweep and the top solve. */
typedef struct ttn_pos_stats_t {
  double energy, lam;     /* as ttn_pos_energy                                  */
  double flops_sweep;     /* product flops of the last ttn_pos_sweep: every node's
                             products, the polar updates' and the top solve's    */
  double bytes_sweep;     /* product bytes of the same (each operand read once,
                             each result written once)                           */
  double lanczos_resid;   /* ||H v - lambda v|| after the last top solve          */
  int n_levels;
  int top_converged;      /* 1 when the last top solve met its target            */
} ttn_pos_stats_t;
ttn_status ttn_pos_stats(ttn_pos_handle h, ttn_pos_stats_t* out);
/* Event timing of the handle's launches by contraction class and kernel, as
 * ttn_profile / ttn_profile_read (same entry layout and warnings). */
ttn_status ttn_pos_profile(ttn_pos_handle h, int enable);
ttn_status ttn_pos_profile_read(ttn_pos_handle h, ttn_profile_entry* out, int max_entries, int* n_out);
/* Replaces a block from the host: TTN_POS_W (level >= 1) the isometries of a
 * layer, node-major, after which every level from it up is ascended again;
 * TTN_POS_TOP the top tensor (chi_{n-1}^2 doubles), not solved again.  The
 * isometries are taken as given (rows are not checked for orthonormality).
 * TTN_EINVAL for another kind or a level outside [1, n). */
ttn_status ttn_pos_set(ttn_pos_handle h, int what, int level, const double* host);
ttn_status ttn_pos_free(ttn_pos_handle h);

/* ------------------------------------------------------------------------
 * Complex tensors: Hamiltonians with complex matrix elements (the paper's
 * method for real tensors, Secs. II.C and III, with every transpose a
 * conjugate transpose).  A uniform network (one isometry per layer, as
 * ttn_init), float64 complex arithmetic throughout.  Conventions: a level
 * tau basis state is |a> = sum_{l,r} w[a; l, r] |l>|r> with rows of w
 * orthonormal in the Hermitian sense; operators ascend as
 * O'[a, a'] = sum conj(w[a; x]) (O w)[a'; x]; the state is
 * sum v[al, be] |al>|be>; the descended matrices pair with operators element
 * by element, rho[a, a'] = <conj(c_a) c_a'> (the transpose of the usual
 * density matrix).  A sweep (Sec. IV): layers bottom-up, each updated to
 * w = -U V^H for its environment Env = U S V^H (Sec. III.B), then v as the
 * lowest eigenvector of the Hermitian top Hamiltonian (Lanczos on its real
 * embedding; its global phase is not fixed).
 *
 * Complex arrays cross this boundary interleaved: (re, im) pairs of
 * doubles, row-major, the layout of C99 double complex and of numpy's
 * complex128.
 * ------------------------------------------------------------------------ */
typedef struct ttn_cplx_ctx* ttn_cplx_handle;

typedef struct ttn_cplx_config {
  int L, d, chi, D;   /* as ttn_config                                         */
  const double* h1;   /* host d*d complex (interleaved), Hermitian             */
  const double* A;    /* host D*d*d complex; B likewise.  The two-site term
                         1/2 (h1 x I + I x h1) + sum_k A_k x B_k must be
                         Hermitian                                            */
  const double* B;
  double shift;       /* NaN: the largest eigenvalue of the bond term          */
  int ly;             /* spins per effective site                             */
  unsigned long long seed; /* start vector of the first top solve when v0 is
                         NULL (counter-based Gaussian real and imaginary
                         parts)                                               */
  const double* const* w0; /* required host array of n-1 pointers: w0[tau-1]
                         is layer tau's chi_tau x chi_{tau-1} x chi_{tau-1}
                         complex isometry                                     */
  const double* v0;   /* optional host chi_{n-1}^2 complex start vector       */
  int krylov, restarts;  /* as in ttn_config, 0: 24, 8                         */
  double lanczos_tol;    /* as in ttn_config, 0: 1e-12                         */
} ttn_cplx_config;

/* Workspace: two planes (real, imaginary) of the network's complex arrays
 * (isometries, operators and descended matrices of every level, a
 * contraction's intermediates, about (3 + 3D) times the largest isometry),
 * and the polar update's buffers for the real embedding of an environment
 * (five times four times the largest isometry).  Errors as
 * ttn_workspace_bytes; TTN_EINVAL when w0 or one of its layers is NULL, when
 * h1 or the bond term is not Hermitian. */
ttn_status ttn_cplx_workspace_bytes(const ttn_cplx_config* cfg, size_t* bytes);
/* Copies the inputs, ascends the operators and solves the top problem.
 * Errors as ttn_init; TTN_WNOCONV when the first top solve ended above its
 * target. */
ttn_status ttn_cplx_init(const ttn_cplx_config* cfg, void* workspace, size_t bytes, void* stream,
                         ttn_cplx_handle* out);
/* nsweeps sweeps (above).  TTN_EHIP / TTN_ENOCONV when a polar Jacobi solve
 * aborted / used its sweep limit; TTN_WNOCONV from the top solver. */
ttn_status ttn_cplx_sweep(ttn_cplx_handle h, int nsweeps);
/* e[0] = top eigenvalue lambda, e[1] = energy per spin of the current state. */
ttn_status ttn_cplx_energy(ttn_cplx_handle h, double* e);
/* rho of every level from 1 up from the current tensors (read back with
 * ttn_cplx_get(TTN_CPLX_RHO)).  Synchronises the stream. */
ttn_status ttn_cplx_descend(ttn_cplx_handle h);
/* The environment of layer tau (1 <= tau < n) from the current tensors
 * (Sec. III.A: rho of level tau and the two-site matrices Rbar, Lbar of the
 * product terms carried up from level tau - 1 through the current layers
 * and down again), into host (chi_tau x chi_{tau-1}^2 complex); the
 * two-site matrices stay readable (TTN_CPLX_RBAR, TTN_CPLX_LBAR).  The state
 * is not changed.  Synchronises the stream. */
ttn_status ttn_cplx_env(ttn_cplx_handle h, int tau, double* host);
/* Copies a complex block to the host (interleaved):
 *   TTN_CPLX_W    (level >= 1) the isometry of layer tau;
 *   TTN_CPLX_OPS  [h, A_1..A_D, B_1..B_D] of a level (chi^2 each; level 0:
 *                 h1 - c I, A, B);
 *   TTN_CPLX_RHO  rho of a level >= 1 as of the last ttn_cplx_descend or
 *                 sweep;
 *   TTN_CPLX_RBAR, TTN_CPLX_LBAR  [Rbar_1..Rbar_D] (Lbar) of the last
 *                 ttn_cplx_env's level (level ignored);
 *   TTN_CPLX_TOP  the top tensor (level ignored). */
enum { TTN_CPLX_W = 0, TTN_CPLX_OPS = 1, TTN_CPLX_RHO = 2, TTN_CPLX_RBAR = 3, TTN_CPLX_LBAR = 4,
       TTN_CPLX_TOP = 5 };
ttn_status ttn_cplx_get(ttn_cplx_handle h, int what, int level, double* host);
/* Replaces a block from the host: TTN_CPLX_W (level >= 1), after which
 * every level from it up is ascended again; TTN_CPLX_TOP, not solved again.
 * TTN_EINVAL for another kind or a level outside [1, n). */
ttn_status ttn_cplx_set(ttn_cplx_handle h, int what, int level, const double* host);
/* Counters of the last sweep and top solve. */
typedef struct ttn_cplx_stats_t {
  double energy, lam;     /* as ttn_cplx_energy                                 */
  double flops_sweep;     /* real flops of the last sweep's products (a complex
                             product is four real ones of its shape)            */
  double bytes_sweep;     /* their bytes (each operand read once, each result
                             written once)                                      */
  double lanczos_resid;   /* ||H v - lambda v|| after the last top solve          */
  double ortho_err_max;   /* largest ||W W^H - I||_F of an update since init      */
  double sigma_ratio_min; /* smallest s_min / s_max of an environment since init  */
  int n_levels;
  int top_converged;      /* 1 when the last top solve met its target            */
  long long repairs;      /* layer updates since init whose environment was
                             numerically rank deficient enough that the polar
                             factor of its real embedding, read as a complex
                             matrix, was not an isometry (off by more than
                             1e-10), and was replaced by its own polar factor   */
} ttn_cplx_stats_t;
ttn_status ttn_cplx_stats(ttn_cplx_handle h, ttn_cplx_stats_t* out);
/* Event timing of the handle's launches, as ttn_profile / ttn_profile_read. */
ttn_status ttn_cplx_profile(ttn_cplx_handle h, int enable);
ttn_status ttn_cplx_profile_read(ttn_cplx_handle h, ttn_profile_entry* out, int max_entries, int* n_out);
ttn_status ttn_cplx_free(ttn_cplx_handle h);

/* Bond dimension chi_tau of member b (tau in 0..n-1), or -1. */
int ttn_bond_dim(ttn_handle h, int b, int tau);

/* Thread-local description of the last error. */
const char* ttn_last_error(void);

ttn_status ttn_free(ttn_handle h);

#ifdef __cplusplus
}
#endif
#endif /* TTN_H */
