/*
 * pm.h -- C ABI of the MI355X product-matrix regenerating-code engine.
 *
 * The engine computes, over GF(2^8), the data phase of the product-matrix
 * (PM) regenerating codes of "Fast Product-Matrix Regenerating Codes"
 * (Le Scouarnec, arXiv 1412.3022): encoding with the linearized generator G
 * or the systematic generator G' = [I; G''] (Sections 3.1-3.3), repair of one
 * node from d helpers, and decoding from any k nodes (Section 2).  Every
 * operation is one region matrix product out[r] = XOR_c A[r][c] * in[c] over
 * byte regions, run by hand-written gfx950 kernels.
 *
 * Conventions for every data call:
 *  - A "region set" is R blocks of block_bytes bytes in device memory; block
 *    r starts at base + r * ld.  base must be 16-byte aligned, ld a multiple
 *    of 16 with ld >= block_bytes.  block_bytes may be any value >= 1.
 *  - Input and output region sets must not overlap (PM_EINVAL).
 *  - Calls only enqueue work on `stream` (a hipStream_t, NULL = the default
 *    stream) and return; the caller owns every buffer and must keep it alive
 *    until the stream has passed the call.  Host-side matrix construction for
 *    a new failure pattern runs synchronously inside the call (the paper's
 *    "initialization" phase, Section 4) and is cached in the code object.
 *  - Errors come back as a pm_status; nothing is thrown across the ABI.
 *    PM_EHIP means a HIP call failed (its message: pm_last_hip_error()).
 *  - A pm_code is immutable after creation apart from internal caches that
 *    are locked; it may be used from several host threads and streams at
 *    once.  The device copy of its tables is made on first use per device.
 *
 * Field: GF(2^8) with polynomial x^8+x^4+x^3+x^2+1 (0x11D) and generator 2,
 * the default field of GF-Complete that the paper uses (Section 3.3).
 */
#ifndef PM_H
#define PM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *pm_stream; /* same object as hipStream_t */

typedef enum {
    PM_OK = 0,
    PM_EINVAL = -1,        /* bad argument: ids, sizes, alignment, aliasing */
    PM_EUNSUPPORTED = -2,  /* parameters outside the constructions */
    PM_ESINGULAR = -3,     /* helper set / node set cannot repair / decode */
    PM_ENOMEM = -4,        /* host or device allocation failed */
    PM_EHIP = -5,          /* a HIP runtime call failed */
    PM_EBUSY = -6,         /* a queue is full; retry later */
    PM_ENOTREADY = -7,     /* the operation has not been prepared on this device
                              (entry points that allocate nothing) */
    PM_ELIMIT = -8         /* beyond a fixed size limit (the static scratch of
                              pm_decode_specific_noalloc) */
} pm_status;

typedef enum {
    PM_MSR = 0,  /* minimum-storage: alpha = d-k+1, d = 2k-2 (Section 2) */
    PM_MBR = 1,  /* minimum-bandwidth: alpha = d (Section 2) */
    PM_RS = 2    /* Reed-Solomon baseline, Vandermonde, systematic (Section 4) */
} pm_kind;

typedef enum {
    PM_VANILLA = 0,  /* Vandermonde Psi of the seminal construction (Section 3.3) */
    PM_SPARSE = 1    /* identity-over-Cauchy Psi proposed by the paper (Section 3.3) */
} pm_construction;

typedef struct {
    uint32_t w;            /* field width: 8, or 16 for the sparse PM-MSR code
                              over GF(2^16) (below) */
    uint32_t k, d, n;      /* MSR: d = 2k-2, n >= d+1 (sparse: n in {2k-1, 2k});
                              MBR: k <= d <= n-1; RS: d ignored, k < n; n <= 255 */
    int32_t kind;          /* pm_kind */
    int32_t construction;  /* pm_construction (MSR only) */
    uint32_t systematic;   /* MSR: 1 = encode with G' = G inverse(G~) (Section 3.2),
                              0 = with G.  MBR and RS are always systematic. */
    const uint8_t *x;      /* MSR vanilla only: n distinct evaluation points
                              (host memory, copied), NULL = x_i = g^i */
} pm_params;

/* GF(2^16) codes (w = 16).  Section 3.3 states that the sparse PM-MSR
 * construction, valid for k up to 39 over GF(2^8), is valid for k up to 64
 * over GF(2^16).  Field: x^16 + x^12 + x^3 + x + 1 (0x1100B), g = 2.
 * Only kind PM_MSR with construction PM_SPARSE (n = 2k-1 or 2k, n <= 65535),
 * systematic or not; others give PM_EUNSUPPORTED.  A block holds 16-bit
 * symbols, little-endian (symbol p in bytes 2p and 2p+1), so block_bytes must
 * be even (else PM_EINVAL).  pm_encode, pm_repair_helper, pm_repair_newcomer
 * and pm_decode run on the GF(2^16) region kernel with the same arguments
 * as for w = 8; pm_prepare builds the operation's matrix, generates and
 * compiles its bit-sliced kernel when the matrix is under the size limit
 * (*specialized = 1; blocks of at least 4096 bytes then run on it) and stages
 * both on the device.  A matrix past one kernel's limit and within two (the
 * k = 16 encode, the k = 8 decode from the parity nodes) gets two kernels
 * over halves of its rows, compiled on two threads (about a minute of
 * hipRTC for the k = 16 encode) and run side by side: the second on an
 * internal stream that waits for the caller's stream, which then waits for
 * it.  That internal stream is shared by all calls on the device: while one
 * thread captures such a call into a graph, other threads should not make
 * such calls until the capture ends.  The specific decoder's passes get one
 * kernel at most.  pm_code_matrix writes two bytes per entry,
 * little-endian (cap counts bytes).  pm_decode_specific (and its workspace,
 * factor and pm_prepare forms) runs the specific PM-MSR decoder's passes on
 * the GF(2^16) kernel; pm_decode_specific_factor writes two bytes per entry.
 * pm_decode_matrix(es), pm_set_variant, pm_autotune_encode, batches and the
 * server take GF(2^8) codes only: PM_EUNSUPPORTED.  Building a systematic
 * code inverts a B x B matrix (B = k(k-1)) on the host, as does each new node
 * set of pm_decode: about 0.5 s and 2 s at k = 40, 5 s and 30 s at k = 64;
 * the specific decode's factors need only alpha x alpha inverses (0.1 s at
 * k = 64). */

typedef struct pm_code pm_code;

/* Build a code: Psi, index matrix L, linearized G (Section 3.1), systematic
 * G' (Section 3.2), the validity check of Section 3.3 (distinct Lambda, every
 * d rows of Psi independent).  Host only: touches no GPU.  *out receives a
 * handle owned by the caller (free with pm_code_destroy).
 * Errors: PM_EINVAL (NULL, shape, unknown kind), PM_EUNSUPPORTED (w other
 * than 8 and 16, or a construction invalid for these parameters),
 * PM_ESINGULAR, PM_ENOMEM. */
pm_status pm_code_create(const pm_params *params, pm_code **out);

/* Free a code and its device tables.  The caller must make sure no stream is
 * still running a call on it. */
void pm_code_destroy(pm_code *code);

/* alpha (blocks per node), beta (= 1, blocks sent per helper), B (message
 * blocks = k Delta), enc_rows (blocks written by pm_encode: the parity rows
 * (n alpha - B for systematic MSR, (n-k) d for MBR, n-k for RS) or all
 * n alpha rows for non-systematic MSR).  Any pointer may be NULL. */
pm_status pm_code_dims(const pm_code *code, uint32_t *alpha, uint32_t *beta,
                       uint32_t *B, uint32_t *enc_rows);

/* Copy a host matrix of the code into host buffer `dst` of `cap` bytes
 * (row-major; two bytes per entry for w = 16), and its shape into *rows,
 * *cols.  which: 0 = Psi (n x d; RS: the n x k generator), 1 = Lambda
 * (1 x n, MSR), 2 = G linearized
 * (n alpha x B), 3 = the generator node contents follow (G' or G),
 * 4 = the encode matrix (enc_rows x B).  PM_EINVAL if cap is too small. */
pm_status pm_code_matrix(const pm_code *code, int which, uint8_t *dst, size_t cap,
                         uint32_t *rows, uint32_t *cols);

/* Where each of the n alpha node blocks lives after pm_encode: map[t] for
 * node t / alpha, block t % alpha, is v < B for message block v (uncoded),
 * or B + r for row r of pm_encode's output.  cap = entries of map. */
pm_status pm_code_node_map(const pm_code *code, int32_t *map, size_t cap);

/* Encode (Section 3.1 / 3.2): out[r] = XOR_c E[r][c] * X[c] for the enc_rows
 * rows E of the encode matrix (G'' for systematic codes, so the message blocks
 * are not rewritten; G for non-systematic MSR).  X: B blocks (device), out:
 * enc_rows blocks (device). */
pm_status pm_encode(const pm_code *code, const uint8_t *X, size_t x_ld, uint8_t *out,
                    size_t out_ld, size_t block_bytes, pm_stream stream);

/* Repair, helper side (Section 2, repair with d helpers sending beta = 1
 * block each): a surviving node projects its alpha blocks onto the failed
 * node's vector -- phi_f for MSR (a unit vector for the first alpha nodes of
 * the sparse code: the helper reads one block, Section 3.3), psi_f for MBR,
 * the block itself for RS.  node: alpha blocks (device); out: 1 block. */
pm_status pm_repair_helper(const pm_code *code, uint32_t failed, const uint8_t *node,
                           size_t node_ld, uint8_t *out, size_t block_bytes,
                           pm_stream stream);

/* Repair, newcomer side: from the d helper blocks (recv, in the order of
 * helpers[], device) rebuild the alpha blocks of node `failed` (out, device).
 * helpers: d distinct node ids != failed (host array).  MSR uses
 * [I | lambda_f I] inverse(Psi_H), MBR inverse(Psi_H), RS row f of G times
 * inverse(G_H) with d = k.  PM_ESINGULAR when Psi_H is singular. */
pm_status pm_repair_newcomer(const pm_code *code, uint32_t failed, const uint32_t *helpers,
                             const uint8_t *recv, size_t recv_ld, uint8_t *out,
                             size_t out_ld, size_t block_bytes, pm_stream stream);

/* Repair of node `failed` in two steps on one stream (Section 2: each of
 * the d helpers sends beta = 1 block, the newcomer solves for its alpha
 * blocks): the d helper projections as one launch of the multi-set
 * bit-sliced kernel over all helpers, then the newcomer's solve.
 * helper_nodes: host array of d device pointers, helper j's alpha blocks at
 * helper_nodes[j] + a * node_ld, in the order of helpers[] (d distinct node
 * ids != failed, host).  workspace (device, 16-byte aligned, at least
 * pm_repair_workspace bytes, not overlapping any other region) receives the
 * d helper blocks -- the bytes the helpers would send over the network --
 * followed by the projections' launch list, which a small kernel writes
 * there in stream order.  out: the alpha rebuilt blocks.  The one-launch
 * projection needs the helper vector's multi-set kernel (pm_prepare op 5,
 * which also prepares the newcomer) and blocks of at least 2048 bytes;
 * otherwise each projection is its own launch.  Same bytes as
 * pm_repair_helper for every helper followed by pm_repair_newcomer; same
 * errors. */
pm_status pm_repair_workspace(const pm_code *code, size_t block_bytes, size_t *bytes);
pm_status pm_repair(const pm_code *code, uint32_t failed, const uint32_t *helpers,
                    const uint8_t *const *helper_nodes, size_t node_ld, uint8_t *workspace,
                    size_t workspace_bytes, uint8_t *out, size_t out_ld, size_t block_bytes,
                    pm_stream stream);

/* Decode (Section 2: X = inverse(G~) Y~): from k distinct nodes (host array
 * `nodes`) whose k alpha blocks are in Y (node-major, in the order of
 * nodes[], device), rebuild the B message blocks X (device).  Message blocks
 * found uncoded in Y are copied, the rest computed (the lazy decoding of
 * Section 3.1).  For MBR the first B independent received rows are used. */
pm_status pm_decode(const pm_code *code, const uint32_t *nodes, const uint8_t *Y,
                    size_t y_ld, uint8_t *X, size_t x_ld, size_t block_bytes,
                    pm_stream stream);

/* Specific PM-MSR and PM-MBR decoding: the seminal paper's data-collector
 * algorithms (Section 2), which the paper's Section 4 finds faster than the
 * linearized decode for large k (MSR: Section 4.1; MBR: its MBR
 * subsection, k >= 7).  Same nodes, Y and X as pm_decode; the result is the
 * same bytes.  It runs as region products with small sparse matrices
 * instead of the dense B x B inverse.  PM-MSR: (0) Z_ij = y_i . phi_j for
 * every ordered pair of the k nodes, from node i's blocks; (1) P_ij and
 * Q_ij of every pair from Z_ij and Z_ji; (2) phi_i^t S1 and phi_i^t S2 for
 * alpha of the nodes by alpha x alpha solves; (3) S1 and S2, i.e. the
 * message symbols; and for systematic codes (4) their re-encoding into the
 * data blocks.  PM-MBR (M = [[S, T], [T^t, 0]], Psi = [Phi, Delta]):
 * (0) T = inverse(Phi_K) times the last d - k blocks of the nodes, beside
 * copies of their first k blocks; (1) the message symbols: T, and S from
 * the first k blocks and Delta_K T^t.  Intermediates go to `workspace`
 * (device, 16-byte aligned, at least pm_decode_specific_workspace bytes,
 * not overlapping Y or X); the library allocates nothing.  PM_EUNSUPPORTED
 * for RS.  Passes use the bit-sliced kernels once compiled (pm_prepare
 * op 4). */
pm_status pm_decode_specific_workspace(const pm_code *code, size_t block_bytes, size_t *bytes);
pm_status pm_decode_specific(const pm_code *code, const uint32_t *nodes, const uint8_t *Y, size_t y_ld,
                             uint8_t *X, size_t x_ld, size_t block_bytes, uint8_t *workspace,
                             size_t workspace_bytes, pm_stream stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * specific decode as pm_decode_specific, same arguments minus the workspace,
 * with the intermediates in a fixed scratch array that the library's code
 * object holds on every device it is loaded on (128 MiB per device, kept
 * until the process ends).  It calls no hipMalloc, hipFree, hipRTC or module
 * load: the node list must have been prepared on the current device first
 * with pm_prepare(code, 4, 0, nodes, 0, ...), which also looks up the
 * scratch's device address there; otherwise PM_ENOTREADY.  PM_ELIMIT when
 * the workspace that pm_decode_specific_workspace reports for block_bytes
 * exceeds 128 MiB.  GF(2^8) codes only (PM_EUNSUPPORTED for w = 16 and RS).
 * Every call on a device shares that device's scratch and it keeps the last
 * call's contents (each pass overwrites what it reads later, so nothing
 * needs clearing): calls that overlap in time on one device -- on different
 * streams, or from different threads -- race and must be serialized by the
 * caller (one stream, or events). */
pm_status pm_decode_specific_noalloc(const pm_code *code, const uint32_t *nodes, const uint8_t *Y, size_t y_ld,
                                     uint8_t *X, size_t x_ld, size_t block_bytes, pm_stream stream);
/* The factor of pass `which` (0..4 above; factor 4 has 0 rows for
 * non-systematic PM-MSR codes, factors 2..4 for PM-MBR) for nodes, host
 * row-major, cap bytes at dst (dst may be NULL to query rows and cols).
 * PM-MSR: their product F4 F3 F2 F1 F0 is the linearized decode matrix of
 * pm_decode.  PM-MBR: F1 F0 (B x k d) reads all k d node blocks and is a
 * left inverse of the generator rows of those blocks. */
pm_status pm_decode_specific_factor(const pm_code *code, const uint32_t *nodes, int which, uint8_t *dst,
                                    size_t cap, uint32_t *rows, uint32_t *cols);

/* Host init of pm_decode for one node set (Section 2: X = inverse(G~) Y~):
 * the B x B decode matrix it applies, row-major into host `D` (cap >= B*B
 * bytes; may be NULL), and in host `kept` (B entries; may be NULL) the
 * indices, among the k alpha received blocks, of the blocks it reads.
 * Built once per node set and kept with the code, as pm_decode does.
 * PM_EINVAL for a bad node list, PM_ESINGULAR if undecodable. */
pm_status pm_decode_matrix(const pm_code *code, const uint32_t *nodes, uint8_t *D, size_t cap, uint32_t *kept);

/* GPU-side init: batched Gauss-Jordan elimination over GF(2^8), one
 * work-group per problem.  The paper reports the initialization (building
 * and inverting the per-failure-pattern matrices) apart from the data phase
 * and finds that it dominates for small objects (Section 4); this computes
 * the decode matrices of `count` node sets at once.  node_sets: device,
 * count x k node ids.  For set p, D + p*d_stride (device, d_stride >= B*B)
 * receives the B x B row-major matrix that pm_decode applies for that set
 * (Section 2: X = inverse(G~) Y~): the inverse of the generator rows of the
 * first B independent blocks, in order, among the set's k alpha blocks
 * (node-major; for MSR and RS all of them, for MBR B of the k d); and
 * kept + p*B (device, may be NULL) receives their indices among those
 * blocks.  status[p] (device) = PM_OK, PM_EINVAL (a node id >= n or
 * repeated) or PM_ESINGULAR (rank < B); D of a failed set is zero.
 * Asynchronous on `stream`; the first call on a device also uploads the
 * generator, which the code keeps.  PM_EUNSUPPORTED when a problem's
 * B x 2B bytes of elimination state exceed one work-group's LDS (PM-MBR
 * with k = 16 on MI355X). */
pm_status pm_decode_matrices(const pm_code *code, const uint32_t *node_sets, uint32_t count, uint8_t *D,
                             size_t d_stride, uint32_t *kept, int32_t *status, pm_stream stream);

/* The same elimination on caller matrices: the inverses of `count` m x m
 * matrices over GF(2^8).  A: device, matrix p at A + p*a_stride with rows
 * a_ld apart; Ainv: device, p at Ainv + p*inv_stride with rows inv_ld
 * apart (Ainv may equal A with the same layout; distinct problems must not
 * overlap).  status[p] (device) = PM_OK or PM_ESINGULAR (inverse zero).
 * Asynchronous on `stream`.  PM_EINVAL for bad sizes or strides,
 * PM_EUNSUPPORTED when m x 2m bytes exceed one work-group's LDS. */
pm_status pm_gf_invert_batch(const uint8_t *A, size_t a_ld, size_t a_stride, uint32_t m, uint32_t count,
                             uint8_t *Ainv, size_t inv_ld, size_t inv_stride, int32_t *status,
                             pm_stream stream);

/* The region engine itself (the constant-times-region multiply-XOR of the
 * paper's Section 4, batched over a matrix): out[r] = XOR_c A[r][c] * in[c]
 * for a host row-major rows x cols matrix A.  Tables are cached by content. */
pm_status pm_apply(const uint8_t *A, uint32_t rows, uint32_t cols, const uint8_t *in,
                   size_t in_ld, uint8_t *out, size_t out_ld, size_t block_bytes,
                   pm_stream stream);

/* Kernel variant for one operation of a code (set by the autotuner or the
 * caller).  op: 0 encode, 1 repair helper, 2 repair newcomer, 3 decode,
 * 4 pm_apply (global).  rows_per_group in {4, 8, 16}: output rows held in
 * registers per work unit; dwords_per_lane in {2, 4} (8 or 16 bytes per lane
 * per source block), plus 10 to stage the coefficient tables in LDS instead
 * of reading them through the scalar cache (12, 14), plus 20 for the
 * software-pipelined kernel that loads every column of the next work unit
 * while multiplying the current one (22, 24; row groups of up to 16
 * columns, others fall back to the plain loop).  dwords_per_lane 32 (with
 * rows_per_group 8): the bit-sliced kernel -- the matrix compiled at first
 * use (hipRTC, a few seconds, cached per matrix and device) into a
 * straight-line XOR network over bit planes (Section 4.1's bit-matrix
 * view); blocks shorter than 2048 bytes and matrices whose network exceeds
 * the size limit run the table kernel with 4 dwords per lane instead.  A
 * hipRTC failure is reported as PM_EHIP.  0, 0 restores the default: the
 * bit-sliced kernel when the operation's matrix has one compiled (by
 * pm_prepare, pm_autotune_encode or a call under variant 32) and the block
 * is at least 2048 bytes; else, for a dense matrix (at most 512 columns;
 * its rows that are not one input block times 1 span at least 64 x 64
 * entries, a third or more of them nonzero) too large to specialize, the
 * matrix-core kernel on those rows, the other rows copied first by the
 * table kernel (dwords_per_lane 40 with
 * rows_per_group 8 selects it explicitly: the matrix's GF(2) expansion, 8
 * rows x 8 columns of bits per coefficient, multiplied with the input bits
 * on v_mfma with 4-bit float operands and reduced to parities, the
 * bit-matrix view of Section 4.1 on the matrix cores; for more than 512
 * columns, or input blocks reaching past 4 GiB from the first, the table
 * kernel runs instead); else the table kernel with the cost-model rows per
 * group and 2 dwords per lane.  The default never compiles by itself.
 * Every variant gives the same bytes.  PM_EINVAL for other values. */
pm_status pm_set_variant(pm_code *code, int op, uint32_t rows_per_group,
                         uint32_t dwords_per_lane);

/* Init phase of one operation, kept apart from the data phase as the
 * paper's evaluation separates them (Section 4): builds the operation's
 * matrix (op 0 encode, 1 repair helper, 2 repair newcomer, 3 decode, 4 the
 * passes of pm_decode_specific, 5 both steps of pm_repair -- the helper
 * projection's multi-set kernel and the newcomer's; failed and ids as for
 * those calls, ids on the host) and, under the default or the
 * bit-sliced variant, generates its bit-sliced kernel and compiles it with
 * hipRTC (seconds; no GPU needed; a no-op when already compiled): the
 * single-set form that the calls above use, or with PM_PREPARE_BATCHED in
 * flags the multi-set form that batches and the server use.  With a GPU
 * present it also uploads the operation's tables and loads the kernel on
 * the current device, so the first data call does neither.  *specialized
 * (may be NULL) = 1 when that kernel is ready, 0 when the table kernel will
 * run (matrix over the size limit, or an explicit table variant).
 * PM_EINVAL for bad ids or flags, PM_EHIP if hipRTC fails. */
#define PM_PREPARE_BATCHED 1u
pm_status pm_prepare(pm_code *code, int op, uint32_t failed, const uint32_t *ids, uint32_t flags,
                     int *specialized);

/* Autotuner for encode: times every kernel variant on the caller's buffers
 * (X, out as for pm_encode; reps launches each, HIP events on `stream`),
 * keeps the fastest for this code and reports it.  Synchronous: returns after
 * the timing runs; out holds a valid encoding afterwards. */
pm_status pm_autotune_encode(pm_code *code, const uint8_t *X, size_t x_ld, uint8_t *out,
                             size_t out_ld, size_t block_bytes, uint32_t reps, pm_stream stream,
                             uint32_t *best_rows_per_group, uint32_t *best_dwords_per_lane);

/* ---- Batched launches (project addition beyond the paper) ----------------
 * Many independent operations -- objects of different sizes and codes,
 * encode, repair and decode mixed -- run as one persistent work-list launch
 * per row-group size, with the waves of the whole GPU pulling (item, row
 * group, byte tile) units from per-XCD queues.  Items of at least 2048 bytes
 * whose matrix has a compiled multi-set bit-sliced kernel (pm_prepare with
 * PM_PREPARE_BATCHED, or PM_BATCH_SPECIALIZE below) run instead as one
 * launch of that kernel per matrix.  The plan fixes every pointer and size;
 * a run only enqueues. */
typedef struct {
    const pm_code *code;
    int32_t op;            /* 0 encode, 1 repair helper, 2 repair newcomer, 3 decode */
    uint32_t failed;       /* op 1, 2: the failed node */
    const uint32_t *ids;   /* op 2: d helper ids; op 3: k node ids (host, read
                              during pm_batch_plan only); NULL otherwise */
    const uint8_t *in;     /* device region set, as for the single calls */
    size_t in_ld;
    uint8_t *out;
    size_t out_ld;         /* ignored for op 1 (one output block) */
    size_t block_bytes;
} pm_batch_item;

typedef struct pm_batch pm_batch;

#define PM_BATCH_GRAPH 1u  /* capture the launches in a HIP graph on the first
                              run and replay it afterwards */
#define PM_BATCH_SPECIALIZE 2u  /* compile, during the plan, the multi-set
                                   bit-sliced kernel of every matrix that has
                                   an item of >= 2048 bytes (seconds per new
                                   matrix, about 30 s for the k = 16 encode) */

/* Resolve every item (building repair / decode matrices as needed), check
 * its regions as the single calls do, and upload the work lists.  Blocks
 * until the uploads land.  The items array is not kept. */
pm_status pm_batch_plan(const pm_batch_item *items, size_t n, uint32_t flags, pm_batch **out);

/* Tile width of the work lists: dwords_per_lane 2 or 4 (8 or 16 bytes per
 * lane per block) for the size class with rows_per_group rows (0 = all). */
pm_status pm_batch_set_variant(pm_batch *batch, uint32_t rows_per_group, uint32_t dwords_per_lane);

/* Autotuner: times each tile width per size class of the table work lists
 * and, for each matrix's bit-sliced multi-set launch, half, all and twice its
 * resident work-group slots (reps runs each, HIP events on `stream`), keeps
 * the fastest of each and reports the last table class's tile width.
 * Synchronous; overwrites the items' outputs with valid results. */
pm_status pm_batch_autotune(pm_batch *batch, uint32_t reps, pm_stream stream,
                            uint32_t *best_dwords_per_lane);

/* Enqueue all items on `stream`.  Runs of one batch share its queue heads,
 * so they must be ordered (one stream, or events between streams). */
pm_status pm_batch_run(pm_batch *batch, pm_stream stream);

/* Work units (item x row group x wave tile) and launches of a plan (table
 * size classes plus bit-sliced matrices). */
pm_status pm_batch_info(const pm_batch *batch, uint64_t *units, uint32_t *size_classes);

/* Free a plan; no run of it may still be in flight. */
void pm_batch_destroy(pm_batch *batch);

/* ---- Served mode (project addition beyond the paper) ---------------------
 * Continuous batching of requests under an HBM budget.  The server owns one
 * device arena of hbm_budget_bytes; a request is admitted (in arrival order)
 * once the arena can hold its result (and, for repair, its d helper blocks),
 * then runs inside a micro-batch on one of `streams` streams.  Requests that
 * arrive while earlier micro-batches run are admitted into the next free
 * stream, so their work overlaps on the GPU.  A result stays in the arena
 * until pm_server_release.  Operations of at least 2048 bytes whose matrix
 * has a compiled multi-set bit-sliced kernel (pm_prepare with
 * PM_PREPARE_BATCHED, before submitting) run on it, one launch per matrix
 * per micro-batch phase; the rest on the table work lists.  The server never
 * compiles by itself. */
typedef enum { PM_REQ_ENCODE = 0, PM_REQ_REPAIR = 1, PM_REQ_DECODE = 2 } pm_request_op;

typedef struct {
    int32_t op;                          /* pm_request_op */
    const pm_code *code;
    uint32_t failed;                     /* repair: the failed node */
    const uint32_t *ids;                 /* repair: d helper ids; decode: k node ids
                                            (host, copied at submit) */
    const uint8_t *in;                   /* encode: X (B blocks); decode: the k alpha
                                            received blocks, node-major (device) */
    size_t in_ld;
    const uint8_t *const *helper_nodes;  /* repair: d device pointers, each to the
                                            alpha blocks of one helper node (host
                                            array, copied at submit) */
    size_t node_ld;
    size_t block_bytes;
    uint64_t tag;                        /* returned in the completion */
} pm_request;

typedef struct {
    uint64_t ticket, tag;
    int32_t status;
    uint8_t *out;          /* result blocks in the arena (device), valid until released */
    size_t out_ld;
    uint32_t out_blocks;   /* encode: enc_rows; repair: alpha; decode: B */
    uint64_t t_submit_ns, t_admit_ns, t_done_ns;   /* steady clock */
} pm_completion;

typedef struct {
    uint64_t hbm_budget_bytes;  /* device bytes for the arena (admitted results +
                                   repair scratch) and the kernel tables */
    uint32_t streams;           /* micro-batches in flight at once (1..16) */
    uint32_t max_batch;         /* requests per micro-batch */
    uint32_t queue_cap;         /* pending requests before submit returns PM_EBUSY */
    uint32_t dwords_per_lane;   /* tile width of the work lists: 2 or 4 (0 = 2) */
    uint64_t table_reserve_bytes;  /* part of the budget kept for the device
                                      copies of kernel tables (pm_table_bytes);
                                      0 = budget / 32, at least 16 MiB.  The
                                      arena is the rest. */
    uint64_t max_batch_bytes;   /* result and scratch bytes per micro-batch
                                   (0 = no limit): admission closes a
                                   micro-batch before a request would take it
                                   past this (a micro-batch always takes at
                                   least one request), so large requests do
                                   not hold the small ones behind them for
                                   long */
} pm_server_cfg;

typedef struct {
    uint64_t completed, batches, pending, arena_used, arena_high_water;
    uint32_t max_concurrent_batches;   /* most micro-batches in flight at once */
    uint32_t pad;
    uint64_t failed;                   /* requests completed with an error status */
    uint64_t arena_bytes;              /* arena size (budget minus the table reserve) */
    uint64_t table_reserve_bytes;
    uint64_t table_bytes_high;         /* most table bytes seen after a micro-batch's
                                          uploads (pm_table_bytes, all codes) */
    uint64_t launch_host_ns;           /* scheduler time spent packing, uploading
                                          and enqueuing micro-batches */
} pm_server_stat;

typedef struct pm_server pm_server;

/* Allocate the arena, streams and staging buffers; start the scheduler
 * thread (on the calling thread's current device).  Kernel tables that the
 * work lists read count against the budget: before a micro-batch uploads
 * tables that would take pm_table_bytes() past the reserve, the scheduler
 * evicts least recently used failure patterns not in use (a device-wide
 * synchronization); if the tables its own requests need still do not fit,
 * those requests complete with PM_ENOMEM.  PM_EINVAL when the reserve
 * leaves no arena. */
pm_status pm_server_create(const pm_server_cfg *cfg, pm_server **out);

/* Queue a request (thread-safe).  Resolves its matrices (building a repair or
 * decode matrix for a new failure pattern here), checks its regions and
 * returns a ticket.  PM_EBUSY when queue_cap requests are pending; PM_ENOMEM
 * when its result can never fit the arena.  Input buffers must stay valid
 * until its completion is polled. */
pm_status pm_server_submit(pm_server *srv, const pm_request *req, uint64_t *ticket);

/* Move up to cap finished requests into out[]; *n_done = how many. */
pm_status pm_server_poll(pm_server *srv, pm_completion *out, size_t cap, size_t *n_done);

/* Give a finished request's arena space back. */
pm_status pm_server_release(pm_server *srv, uint64_t ticket);

pm_status pm_server_stats(pm_server *srv, pm_server_stat *st);

/* Load driver: submit reqs[i] at arrival_ns[i] after the call starts (spin
 * waiting, retrying while the queue is full), collect every completion into
 * out[i], and release each result at once unless flags has PM_REPLAY_KEEP.
 * Returns when all n requests have completed. */
#define PM_REPLAY_KEEP 1u
pm_status pm_server_replay(pm_server *srv, const pm_request *reqs, const uint64_t *arrival_ns,
                           size_t n, uint32_t flags, pm_completion *out);

/* Stop the scheduler after the micro-batches in flight finish; free all. */
void pm_server_destroy(pm_server *srv);

/* ---- Caches of per-failure-pattern state ----------------------------------
 * The initialization phase of a repair or decode (Section 4: built once per
 * failure pattern) is cached in the code object: the helper, newcomer and
 * decode matrices, the specific-decode factors, their kernel programs, the
 * device copies of their tables and their compiled kernels.  Each of these
 * caches holds at most `entries` patterns (default 256); beyond that the
 * least recently used pattern not in use (by a batch plan, a queued server
 * request or a call in progress) is evicted.  An evicted pattern's device
 * memory is freed only once no launch can still read it: after a
 * device-wide synchronization, which the library runs when evicted patterns
 * hold more than 64 MiB, and in pm_cache_release.  The pm_apply cache (keyed
 * by matrix content, all codes) holds 256 matrices the same way.
 * PM_EINVAL for entries == 0. */
pm_status pm_code_set_cache_limit(pm_code *code, uint32_t entries);

/* Synchronize the device and free every evicted pattern that nothing still
 * uses.  Must not be called while a stream of this thread is being
 * captured into a graph. */
pm_status pm_cache_release(void);

/* Device bytes held by the per-matrix kernel tables and matrix-core
 * operands of every code on every device (evicted patterns not yet freed
 * included; not the fixed 8 MiB GF(2^16) field table, which a GF(2^16) code
 * uploads once per device and nothing evicts); the server keeps this within
 * its table reserve. */
size_t pm_table_bytes(void);

/* Failure injection for tests of the error paths: the next `count` uploads
 * of kernel tables to the device fail with PM_ENOMEM, before allocating. */
pm_status pm_debug_fail_uploads(uint32_t count);

/* Message of the last failing HIP call on this thread ("" if none). */
const char *pm_last_hip_error(void);
const char *pm_status_string(pm_status st);

#ifdef __cplusplus
}
#endif
#endif /* PM_H */
