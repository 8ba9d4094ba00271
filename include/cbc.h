/*
 * cbc.h -- C ABI of the MI355X (gfx950) Cholesky-based compression library.
 *
 * The library applies a tree tensor network operator (TTNO; an MPO on a chain) to a tree tensor
 * network state (TTNS; an MPS on a chain) and compresses the product to a target bond dimension,
 * following Milbradt, Sun, Mendl, Gray, Chan, "Efficient Application of Tensor Network Operators to
 * Tensor Network States" (arXiv 2601.19650):
 *   - the problem statement, computing O|psi> for O and psi given as tree tensor networks
 *     (Sec. I, Eq. abstr_application; Sec. II, Eqs. ttns and ttno);
 *   - the compression of Sec. III A (tensor trains) and Sec. III B (general trees): environment
 *     contractions, truncation of the joined leg to the target dimension, QR on the parent leg and
 *     the environment update, with the output rule closing each subsection;
 *   - the optional tolerance-adaptive bond dimension of Sec. V;
 *   - the naive method of Sec. III C: contract exactly, then compress with truncated SVDs.
 *
 * Data model (Sec. II A-C):
 *   - a rooted tree of n nodes: parent[i] in [0, n) or -1 for exactly one root. The children of i
 *     are the nodes j with parent[j] == i, in increasing j.
 *   - state node i has legs (sigma_i, alpha_parent, alpha_child_1, ..., alpha_child_K) and the
 *     operator node (sigma'_i, sigma_i, beta_parent, beta_child_1, ..., beta_child_K). Tensors are
 *     stored row-major (last leg fastest) as interleaved complex128 (re, im). The root's parent leg
 *     is a trivial leg of dimension 1. A node may have d_i = 1 (no physical leg, Sec. II A).
 *   - all node tensors of one network live in one device buffer; offset[i] is the element offset of
 *     node i (one element = one complex number).
 *
 * Numerics (precision argument):
 *   CBC_PREC_FP64  -- every contraction, Gram matrix, eigensolve and Cholesky factorisation in FP64.
 *   CBC_PREC_MIXED -- contractions in FP32 (complex through real MFMA products, FP32 accumulation);
 *                     Gram matrices are accumulated in FP64, and eigensolves, Cholesky factorisations
 *                     and triangular inverses run in FP64.
 *   Truncation keeps the top-k eigenspace of the FP64 Gram matrix of the joined-leg matrix, which is
 *   the truncated SVD the paper uses, reached through its Gram matrix. The QR on the parent leg is a
 *   shifted Cholesky-QR with two re-orthogonalisation passes (Cholesky-QR3). Pivots that vanish
 *   (rank-deficient input) are dropped, which leaves zero slices on that bond.
 *
 * Ownership: the caller owns all device memory (inputs, workspace, outputs). The library never frees
 * caller memory. A context owns only its plan cache (device offset tables, captured graphs), which is
 * released by cbc_destroy. One context per host thread; a context must not be used concurrently.
 *
 * Streams: calls are stream-ordered and asynchronous on the given hipStream_t (passed as void*;
 * NULL = null stream): every shape is fixed by max_bond before device work, so the output bond
 * dimensions are returned at once and the output tensors are ready when the stream reaches the end
 * of the call. Only the profiling mode (cbc_stats.profile) synchronises the stream. The first call
 * with a given set of buffers on a non-null stream captures the launch sequence into a hipGraph;
 * later calls with the same buffers replay it. If the stream is already being captured by the caller,
 * the kernels are recorded into the caller's graph instead; a call with the same shape must have run
 * once before (it builds the plan and uploads its tables, which a capture cannot record).
 *
 * Errors: every entry point returns a cbc_status; nothing aborts or throws across the ABI. All
 * argument validation happens on the host before any device work is queued. Failures that can only
 * be seen on the device are recorded in a status word in the call's workspace and read, after the
 * call has finished, with cbc_read_report: a factorisation or eigensolve that meets non-finite
 * values (CBC_ENOTPD), or a bounded wait that expired (CBC_ETIMEOUT).
 *
 * Eigensolves (Grams of dimension s): s <= 128 run in one workgroup. Larger Grams of a single
 * instance queued eagerly or in the library's own graphs use a Householder reduction spread over up
 * to 256 workgroups that wait for each other (s <= 1536); the library orders these solves one after
 * another on each device (a device-wide event, across streams and contexts of the process), and
 * their waits are bounded (2 s), so a device shared with other spinning work cannot hang the call:
 * it ends with CBC_ETIMEOUT in the report instead. Batches, calls recorded into a caller's stream
 * capture, cbc_apply_noalloc and Grams above 1536 (up to 2064) use a two-stage reduction (dense to
 * band on FP64 matrix cores, band to tridiagonal in one workgroup) that has no waits between
 * workgroups; nothing is recorded into a caller's capture beyond the call's own kernels.
 */
#ifndef CBC_H
#define CBC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CBC_OK = 0,
  CBC_EINVAL = -1,     /* null pointer, max_bond < 1, tol < 0 or not finite, bad precision */
  CBC_ESHAPE = -2,     /* bad topology (no/two roots, cycle, parent out of range) or dims */
  CBC_ENOMEM = -3,     /* workspace smaller than cbc_query reported, or a context allocation failed */
  CBC_EHIP = -4,       /* a HIP runtime call failed */
  CBC_ENOTPD = -5,     /* reserved: a factorisation failed even after its fallbacks */
  CBC_EUNSUP = -6,     /* valid input outside this build's limits: an eigensolve larger than the
                          solver's limit, or a tensor of 2^31 or more elements */
  CBC_ENOTBUILT = -7,  /* library built without a usable device (no gfx950 GPU visible) */
  CBC_ETIMEOUT = -8    /* device side: a bounded cross-workgroup wait expired (output invalid) */
} cbc_status;

typedef enum { CBC_PREC_FP64 = 0, CBC_PREC_MIXED = 1 } cbc_precision;

typedef struct cbc_ctx cbc_ctx;

/* Tree and dimensions (host arrays, read during the call only). */
typedef struct {
  int32_t n_nodes;
  const int32_t* parent;   /* parent[i], -1 for the root */
  const int32_t* phys;     /* d_i >= 1 */
  const int32_t* chi;      /* state bond of node i to its parent (1 at the root) */
  const int32_t* dop;      /* operator bond of node i to its parent (1 at the root) */
} cbc_tree;

/* A network's node tensors: one device buffer of interleaved complex128, host offset array. */
typedef struct {
  const void* data;        /* device pointer */
  const int64_t* offset;   /* host, n_nodes entries, element offsets into data */
} cbc_tensors;

/* The compressed state. Node i is written at out_offset[i] (from cbc_query) with legs
 * (sigma_i, bond_parent, bond_child_1, ...) as interleaved complex128, packed row-major at the start
 * of its slot; bond[] is written on return. Slots are sized for the largest bonds the call can
 * produce, so node i may use less than out_offset[i+1] - out_offset[i] elements. */
typedef struct {
  void* data;              /* device pointer, at least out_offset[n_nodes] elements */
  const int64_t* offset;   /* host, n_nodes + 1 entries as returned by cbc_query */
  int32_t* bond;           /* host, n_nodes entries: bond of node i to its parent (1 at the root) */
} cbc_out;

/* Kernel classes reported in cbc_stats. */
enum {
  CBC_K_CONTRACT = 0,  /* environment / operator contractions, projections, environment updates */
  CBC_K_GRAM = 1,      /* FP64 Gram matrices (truncation and QR) */
  CBC_K_QRMUL = 2,     /* Q = C^{-1} S products of the Cholesky-QR */
  CBC_K_EIG = 3,       /* truncation eigensolves */
  CBC_K_CHOL = 4,      /* Cholesky factorisations and triangular inverses */
  CBC_K_OTHER = 5,     /* conversions, output writes, fills */
  CBC_K_NCLASS = 6
};

/* Per-call statistics (optional). `profile` is an input: when nonzero the call records a HIP event
 * pair around every kernel on the call's stream and fills ms[] (no hipGraph replay in that mode). */
typedef struct {
  int32_t profile;                   /* in: 1 = time every kernel class with HIP events */
  int32_t n_kernels;                 /* out: kernels launched per call */
  int32_t n_eig;                     /* out: eigensolves performed */
  int32_t max_eig_dim;               /* out: largest Gram matrix that was eigensolved */
  int32_t graph_replayed;            /* out: 1 if the call replayed a cached hipGraph */
  int32_t launches[CBC_K_NCLASS];    /* out: launches per kernel class */
  double flops[CBC_K_NCLASS];        /* out: algorithmic flops per class (8 per complex MAC) */
  double bytes[CBC_K_NCLASS];        /* out: algorithmic bytes moved per class (operands + result) */
  double ms[CBC_K_NCLASS];           /* out: summed kernel time per class (profile mode only) */
} cbc_stats;

/* One truncation of a call (Sec. III A / III B: the joined leg compressed to the target dimension),
 * recorded on the device. */
typedef struct {
  int32_t node;        /* the edge from `node` to its parent is truncated */
  int32_t sweep;       /* 1: subtree environment (Eq. cbc_tree_first_contraction); 2: environment of
                          the rest of the tree (Eqs. tt_cbc_first_contraction,
                          cbc_tree_second_contraction); 0: a truncation of the naive method;
                          3: a basis of the density-matrix method (cbc_apply_dm); 4: a basis of
                          the Zip-Up method (cbc_apply_zipup) */
  int32_t dim;         /* dimension of the Gram matrix that was eigensolved */
  int32_t kmax;        /* directions planned (min(max_bond, Gram dimension)) */
  int32_t kept;        /* directions kept (fewer than kmax only with a tolerance) */
  int32_t flags;       /* bit 0: relative gap at the cut below 1e-8 (ties, Sec. III A is silent) */
  double discarded;    /* discarded weight sum_{j >= kept} lambda_j / sum_j lambda_j (lambda: the Gram's
                          eigenvalues = squared singular values; absolute accuracy ~1e-15) */
  double gap;          /* (lambda_{kept-1} - lambda_kept) / lambda_{kept-1}; 1 if nothing is cut */
} cbc_trunc_record;

/* What a finished call recorded on the device. */
typedef struct {
  int32_t status;          /* out: CBC_OK, CBC_ENOTPD or CBC_ETIMEOUT */
  int32_t dropped_pivots;  /* out: Cholesky pivots dropped by the QR steps (rank-deficient S) */
  int32_t n_trunc;         /* out: truncations the call performed */
  int32_t capacity;        /* in: entries available in trunc (0 with trunc == NULL) */
  cbc_trunc_record* trunc; /* in: host array; the first min(capacity, n_trunc) records are written */
} cbc_report;

/* Create / destroy a context. */
cbc_status cbc_create(cbc_ctx** ctx);
void cbc_destroy(cbc_ctx* ctx);
const char* cbc_status_str(cbc_status s);

/* Autotuning of the contractions (the dense complex contractions of Sec. III: the environment,
 * Gram, projection and QR products), per GEMM shape and batch: the tile shape of the MFMA kernel
 * (32 x 32, 64 x 64 or the pipelined 64 x 64, which accumulates in FP32 only) and the split of the
 * reduction into 1, 2, 4 or 8 chunks. After this call, plans built by the context reserve scratch
 * for the split candidates (cbc_query reports the larger workspace), and the first call of a plan
 * with a new batch times every feasible configuration of each contraction on the call's own
 * operands (three launches each, HIP events on the call's stream, which it waits for), keeps the
 * fastest and records it; the call then computes its result as usual. Calls recorded into a
 * caller's graph capture are not tuned. cache_path (may be NULL or empty) names a text file of
 * earlier choices, one "cbc-gemm" line per shape: it is read now (other lines are skipped) and new
 * choices are appended to it. Returns CBC_EINVAL for a null ctx or a cache file that cannot be
 * opened for appending. */
cbc_status cbc_autotune(cbc_ctx* ctx, const char* cache_path);

/* Sizes for a problem: workspace bytes and the output packing (n_nodes + 1 offsets; the last entry is
 * the total number of complex elements the output buffer must hold). Host only, no device work.
 * `method` is 0 for cbc_apply, 1 for cbc_apply_naive, 2 for cbc_apply_src, 3 for cbc_apply_dm and 4
 * for cbc_apply_zipup. */
cbc_status cbc_query(cbc_ctx* ctx, const cbc_tree* tree, int32_t max_bond, cbc_precision prec,
                     int32_t method, size_t* workspace_bytes, int64_t* out_offset);

/* The output bond dimensions cbc_apply will report (host only, no device work): bond[i] for the
 * edge from node i to its parent, 1 at the root. With tol_on = 0 they are the economy-QR bonds
 * min(environment bond, sigma' x child bonds); with tol_on = 1 every edge keeps its planned
 * environment bond (slices beyond the kept directions are zero). */
cbc_status cbc_plan_bonds(cbc_ctx* ctx, const cbc_tree* tree, int32_t max_bond, int32_t tol_on,
                          int32_t* bond);

/* Planned cost of one call (host only, no device work), for scheduling many problems on one GPU:
 * the workspace split into the part that lives through the whole call (report, environments,
 * converted inputs; it starts the workspace) and the scratch reused from node step to node step
 * (it follows), whose sum is cbc_query's workspace_bytes for the same tol_on; and per kernel class
 * (CBC_K_*) the kernels launched and their algorithmic flops (a complex multiply-add counts 8, a
 * Hermitian Gram half its products, an eigensolve 16/3 s^3 + 8 s^2 k, a Cholesky factorisation
 * with its inverse 8/3 k^3), the same figures cbc_stats reports after the call. `method` as in
 * cbc_query. */
typedef struct {
  size_t persistent_bytes;
  size_t scratch_bytes;
  size_t table_bytes;   /* device memory the context holds for the plan's offset tables once it runs */
  int32_t launches[CBC_K_NCLASS];
  double flops[CBC_K_NCLASS];
} cbc_plan_summary;
cbc_status cbc_plan_info(cbc_ctx* ctx, const cbc_tree* tree, int32_t max_bond, cbc_precision prec,
                         int32_t method, int32_t tol_on, cbc_plan_summary* info);

/* Cholesky-based compression of O|psi> (Sec. III A for chains, Sec. III B for trees).
 * max_bond >= 1 is the target bond dimension (the paper's D-bar); tol >= 0 additionally drops
 * directions whose singular value is at most tol times the largest one at that truncation (tol = 0
 * keeps min(max_bond, rank bound) directions). workspace must hold cbc_query's workspace_bytes. */
cbc_status cbc_apply(cbc_ctx* ctx, const cbc_tensors* ttno, const cbc_tensors* ttns,
                     const cbc_tree* tree, int32_t max_bond, double tol, cbc_precision prec,
                     void* workspace, size_t workspace_bytes, cbc_out* out, void* stream,
                     cbc_stats* stats);

/* cbc_apply with its workspace in two buffers: `workspace` holds what lives through the call (at
 * least cbc_plan_info's persistent_bytes for this tol; the report is read from it as usual) and
 * `scratch` what the node steps reuse (at least scratch_bytes). Calls that run one after another on
 * one stream may share one scratch buffer sized for the largest of them, which is how many problems
 * of different shapes fit on one GPU at once (their persistent parts are small). Calls that may
 * overlap (other streams without an ordering between them) must not share it. Returns CBC_EINVAL
 * for a null scratch and CBC_ENOMEM for a buffer below its size; otherwise as cbc_apply. */
cbc_status cbc_apply_split(cbc_ctx* ctx, const cbc_tensors* ttno, const cbc_tensors* ttns,
                           const cbc_tree* tree, int32_t max_bond, double tol, cbc_precision prec,
                           void* workspace, size_t workspace_bytes, void* scratch,
                           size_t scratch_bytes, cbc_out* out, void* stream, cbc_stats* stats);

/* One problem of a cbc_apply_many call: its own tree, networks, target bond, tolerance, workspace,
 * output and (optional) statistics, with the meanings they have in cbc_apply. */
typedef struct {
  const cbc_tree* tree;
  const cbc_tensors* ttno;
  const cbc_tensors* ttns;
  int32_t max_bond;
  double tol;
  void* workspace;          /* device; see cbc_apply_many for its size */
  size_t workspace_bytes;
  cbc_out* out;
  cbc_stats* stats;         /* may be NULL */
} cbc_problem;

#define CBC_MAX_STREAMS 64

/* `count` independent compressions of different shapes (trees, dimensions, max_bond, tol) in one
 * call, for uneven batches (Sec. III B's sweeps run per problem; problems share nothing but the
 * scratch below). Problem j runs on stream j % nstreams of the context (1 <= nstreams <=
 * CBC_MAX_STREAMS, default priority, created on first use); those streams start after the work
 * queued on `stream` before the call, and `stream` continues only after all problems (event fork
 * and join), so the call is ordered like a kernel on `stream`. Eagerly, each problem replays its own
 * captured graph; inside a caller's capture of `stream` the fork, the problems and the join are
 * recorded into the caller's graph. With scratch == NULL every workspace holds cbc_query's
 * workspace_bytes; otherwise scratch[s] (scratch_bytes[s] bytes) is shared by the problems of stream
 * s, one after another, and each workspace holds the persistent part (cbc_plan_info; as for
 * cbc_apply_split). CBC method, one precision for all. Argument errors are returned before any
 * device work; a problem that fails stops the launches of the rest, and the call still joins its
 * streams into `stream`. Each problem's report is read from its workspace (cbc_read_report). */
cbc_status cbc_apply_many(cbc_ctx* ctx, int32_t count, const cbc_problem* problems,
                          cbc_precision prec, int32_t nstreams, void* const* scratch,
                          const size_t* scratch_bytes, void* stream);

/* A batch of `batch` independent compressions of the same shape (same tree, dimensions, max_bond,
 * tol and precision) in one launch sequence: every kernel runs all instances at once. Instance b's
 * node i is at element b * T + offset[i] of each input buffer, where T is the network's total
 * element count (sum of node sizes), and at b * out_offset[n_nodes] + out_offset[i] of the output;
 * the workspace must hold batch times cbc_query's workspace_bytes. bond[] is shared by all
 * instances. Otherwise as cbc_apply. */
cbc_status cbc_apply_batched(cbc_ctx* ctx, int32_t batch, const cbc_tensors* ttno,
                             const cbc_tensors* ttns, const cbc_tree* tree, int32_t max_bond,
                             double tol, cbc_precision prec, void* workspace,
                             size_t workspace_bytes, cbc_out* out, void* stream,
                             cbc_stats* stats);

/* Naive baseline (Sec. III C, the direct method): contract O|psi> exactly (bonds chi*D), bring it into
 * canonical form toward the root with Cholesky-QR, then truncate every bond with the top-k
 * eigenspace of its Gram matrix in a depth-first sweep from the root. Same arguments as cbc_apply. */
cbc_status cbc_apply_naive(cbc_ctx* ctx, const cbc_tensors* ttno, const cbc_tensors* ttns,
                           const cbc_tree* tree, int32_t max_bond, double tol, cbc_precision prec,
                           void* workspace, size_t workspace_bytes, cbc_out* out, void* stream,
                           cbc_stats* stats);

/* Successive randomised compression (SRC), the randomised counterpart of CBC that Sec. III C
 * describes: one random sketch matrix of size d_i x max_bond per node, combined over nodes by the
 * Khatri-Rao product, replaces the truncated environments of sweeps 1 and 2 (Eqs.
 * cbc_tree_first_contraction, cbc_tree_second_contraction) by exact sketches of the subtree below a
 * node and of the rest of the tree; sweep 3 (Eqs. cbc_tree_third_contraction,
 * cbc_final_contraction) takes each node's new basis from a Cholesky-QR of its sketched columns
 * Y = Z E instead of a QR on the parent leg. Only contractions and QRs: no eigensolve. The sketch of
 * node i acts on its output physical leg: `sketch` holds one complex128 d_i x max_bond row-major
 * matrix per node at element offset sketch->offset[i] of sketch->data (device; packed like the
 * inputs), drawn by the caller (for example complex Gaussian). The new bond of node i is
 * min(max_bond, d_i x its children's new bonds); a node whose rows do not exceed max_bond keeps the
 * identity basis. Workspace from cbc_query with method 2. Single instances, no tolerance. Returns
 * CBC_EINVAL for a null or unpacked sketch; otherwise as cbc_apply (no truncation records). */
cbc_status cbc_apply_src(cbc_ctx* ctx, const cbc_tensors* ttno, const cbc_tensors* ttns,
                         const cbc_tensors* sketch, const cbc_tree* tree, int32_t max_bond,
                         cbc_precision prec, void* workspace, size_t workspace_bytes, cbc_out* out,
                         void* stream, cbc_stats* stats);

/* Density-matrix compression, the method CBC is built from (Sec. III; Tab. time_scal and mem_scal
 * give its cost): sweeps 1 and 2 contract the exact environments of <Phi|Phi>, Phi = O|psi>, on
 * both sides of every bond (legs of both copies of the network: (chi_S D_O)^2 elements per bond), and
 * sweep 3 (as in CBC, Eqs. cbc_tree_third_contraction, cbc_final_contraction) takes each node's
 * basis from the top min(max_bond, rows) eigenvectors of its reduced density matrix Z B Z^H (FP64,
 * through the truncation eigensolver; records with sweep 3). A node whose rows do not exceed
 * max_bond keeps the identity basis. Workspace from cbc_query with method 3. Single instances, no
 * tolerance. Otherwise as cbc_apply. */
cbc_status cbc_apply_dm(cbc_ctx* ctx, const cbc_tensors* ttno, const cbc_tensors* ttns,
                        const cbc_tree* tree, int32_t max_bond, cbc_precision prec, void* workspace,
                        size_t workspace_bytes, cbc_out* out, void* stream, cbc_stats* stats);

/* Zip-Up (Sec. III C; Tab. time_scal and mem_scal give its cost): one sweep, leaves to root, in which
 * each node is compressed on the spot from its own product with the already compressed children,
 * Z = T W prod_c R^{[c]} (Eqs. cbc_tree_third_contraction, cbc_final_contraction), with no environment
 * of the rest of the network: the node's basis is the top min(max_bond, rows) eigenvectors of Z Z^H
 * over its parent bond (the left singular vectors of its unfolding; FP64, through the truncation
 * eigensolver; records with sweep 4), R = Q^H Z carries the rest upward and the root keeps Z. The
 * input state is used in the gauge it is given. A node whose rows do not exceed max_bond keeps the
 * identity basis. Workspace from cbc_query with method 4. Single instances, no tolerance. Otherwise
 * as cbc_apply. */
cbc_status cbc_apply_zipup(cbc_ctx* ctx, const cbc_tensors* ttno, const cbc_tensors* ttns,
                           const cbc_tree* tree, int32_t max_bond, cbc_precision prec,
                           void* workspace, size_t workspace_bytes, cbc_out* out, void* stream,
                           cbc_stats* stats);

/* For callers that cannot allocate device memory (code under stream capture, tight serving loops,
 * harnesses that forbid hipMalloc): cbc_apply without a workspace argument. Its workspace is a
 * static device array of 128 MiB per GPU, held by the library until the process ends; the call
 * copies the plan's offset tables there (first 256-byte-aligned part) and uses the rest as the
 * workspace cbc_query reports. It calls no hipMalloc, hipFree or other allocating routine and
 * launches its kernels directly on `stream` (no graph, no autotuning; truncation eigensolves take
 * the two-stage reduction). Same arguments and results as cbc_apply otherwise. Returns CBC_EUNSUP
 * if the tables and the workspace need more than 128 MiB (for example the 64-site and 31-node
 * workloads fit, the 128-site large-bond one does not), CBC_EINVAL if stats->profile is set.
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU (other streams,
 * other host threads) race. The call's report cannot be read with cbc_read_report. */
cbc_status cbc_apply_noalloc(cbc_ctx* ctx, const cbc_tensors* ttno, const cbc_tensors* ttns,
                             const cbc_tree* tree, int32_t max_bond, double tol, cbc_precision prec,
                             cbc_out* out, void* stream, cbc_stats* stats);

/* Report of the last call that used `workspace` (cbc_apply, cbc_apply_batched or cbc_apply_naive):
 * synchronises `stream` (the call's stream),
 * then copies the status word, the dropped-pivot count and the truncation records from the
 * workspace. For batched calls, `instance_bytes` is the per-instance workspace size (cbc_query's
 * workspace_bytes) and `instance` selects the instance; for single calls pass 0 and 0. Returns
 * CBC_EINVAL for null arguments or a workspace that holds no report, CBC_EHIP if a copy fails, and
 * otherwise the device status (CBC_OK, CBC_ENOTPD or CBC_ETIMEOUT), which is also rep->status. */
cbc_status cbc_read_report(const void* workspace, size_t instance_bytes, int32_t instance,
                           void* stream, cbc_report* rep);

#ifdef __cplusplus
}
#endif
#endif /* CBC_H */
