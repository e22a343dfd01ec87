/*
 * sf.h -- C ABI of the star-forest (SF) communication kernels for AMD
 * MI355X (gfx950).
 *
 * The SF model is the one of "The PetscSF Scalable Communication Layer":
 * a star is one root with zero or more leaves, a star forest is a union of
 * disjoint stars, leaves without a root are holes (Section 3.1, Fig. 1).
 * This library runs one device's share of an SF: every root is local, and
 * the leaves that a would-be neighbour rank owns form one segment of a
 * contiguous leaf buffer (Section 5.1 two-sided lists, Section 5.2 pack /
 * unpack / scatter).  The data-parallel hot path -- the pack/unpack-with-
 * reduction kernels behind SFBcast, SFReduce and SFFetchAndOp -- runs as
 * hand-written HIP kernels on the caller's stream.
 *
 * Conventions for every call:
 *  - Return value: SF_OK (0) on success, a negative sf_error otherwise; no
 *    call aborts the process.  sf_error_string() describes a code.
 *  - Host arguments (ilocal, iremote, opts, items, out-pointers) are read
 *    during the call only, unless a copy mode says otherwise.
 *  - Data arguments (rootdata, leafdata, leafupdate) are DEVICE pointers
 *    owned by the caller, arrays of units (see sf_unit), aligned to the
 *    unit's element size.  They are borrowed from *_begin to the matching
 *    *_end and must not be modified in between (Section 3.2).
 *  - stream is a hipStream_t (NULL = the null stream).  Begin enqueues the
 *    kernels; End is stream-ordered and never blocks the host: results are
 *    visible to later work on the same stream (or after synchronising it).
 *    With the environment variable SF_DEBUG=1, *_begin queries each data
 *    pointer and returns SF_ERR_ARG for memory that is not device memory.
 *  - Device indices are 32-bit: nroots and the leaf space must be < 2^31.
 *  - An SF and its scratch memory may be used by one stream at a time.
 *    Scratch is allocated on an operation's first call and grown when a
 *    later call needs more; outgrown buffers are kept until sf_setup or
 *    sf_destroy.  So calls may be captured into a HIP graph once the same
 *    calls have run eagerly (capture allocates nothing), and such graphs
 *    stay valid until the SF is set up again or destroyed.
 *  - sf_setup uploads the plan to the current device; *_begin returns
 *    SF_ERR_ARG when called with another device current.
 */
#ifndef SF_H
#define SF_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ----------------------------------------------------------------- types */

typedef struct sf_s *sf_t;             /* opaque SF handle (PetscSF, Section 3.1) */
typedef struct sf_batch_s *sf_batch_t; /* opaque batch of SF operations */

/* Root address of a leaf (PetscSFNode{rank, offset}, Section 3.1).  rank is
 * the owner rank in the paper; on one device it is the segment label of the
 * leaf (leaves of one label form one segment).  index is the local root. */
typedef struct {
  int64_t rank;
  int64_t index;
} sf_node;

/* Ownership of ilocal / iremote (PetscCopyMode, Section 3.1). */
typedef enum {
  SF_COPY_VALUES = 0, /* the library copies the arrays */
  SF_USE_POINTER = 1, /* the library borrows them until sf_destroy; caller keeps them unchanged */
  SF_OWN_POINTER = 2  /* not supported: returns SF_ERR_UNSUPPORTED */
} sf_copymode;

/* Element type of a unit.  SF_F64_I32 is the MAXLOC / MINLOC pair
 * struct { double v; int32_t i; int32_t pad; } with a 16-byte extent; pad
 * never affects a result and is never written in the caller's roots or leaves
 * (large SFs copy whole 16-byte leaf units, pad included, into scratch).
 * SF_F16 is IEEE binary16, SF_BF16 bfloat16 (binary32's sign and exponent
 * with 7 fraction bits), both 2 bytes: every SUM / PROD of them is the exact
 * result rounded once to the unit's format (nearest, ties to even), MAX / MIN
 * order -0 < +0.  They take the direct deterministic kernels in every reduce
 * mode (no per-element 16-bit atomics), are not partitioned, and are not
 * accepted by FetchAndOp or in a batch (SF_ERR_UNSUPPORTED). */
typedef enum {
  SF_F64 = 0,
  SF_F32 = 1,
  SF_I32 = 2,
  SF_I64 = 3,
  SF_F64_I32 = 4,
  SF_F16 = 5,
  SF_BF16 = 6
} sf_dtype;

/* A unit is bs contiguous elements of one dtype: the "unit" MPI datatype of
 * Section 3.2.  Ops act per element (MAXLOC / MINLOC: per pair). */
typedef struct {
  int32_t dtype; /* sf_dtype */
  int32_t bs;    /* block size, >= 1 */
} sf_unit;

/* Operation (MPI_Op of Section 3.2, which names the MPI reductions as the
 * ops of Bcast and Reduce).  SUM, MAX, MIN and PROD act on F64, F32, I32,
 * I64 (integers wrap around), F16 and BF16; MAXLOC and MINLOC on F64_I32
 * pairs.  PROD and
 * MINLOC have no native device atomic: they combine through the
 * deterministic kernels in every reduce mode. */
typedef enum { SF_REPLACE = 0, SF_SUM = 1, SF_MAX = 2, SF_MIN = 3, SF_MAXLOC = 4, SF_MINLOC = 5, SF_PROD = 6 } sf_op;

/* How SFReduce combines leaves of a root that has several (Section 5.3 uses
 * atomics when destinations repeat).
 *  AUTO          : the deterministic path (measured as fast as or faster
 *                  than the atomic one); FetchAndOp on FP units and batch
 *                  items with roots of more than 256 leaves use atomics;
 *  ATOMIC        : native atomics, with block-local aggregation of the
 *                  roots of highest degree; on a partitioned SF (below) a
 *                  root whose leaves all fall in one window is updated
 *                  plainly and a root spanning windows takes one native
 *                  atomic per window (FetchAndOp: a returning atomic add);
 *                  FP SUM order is unspecified (PROD, MAXLOC in some
 *                  configurations and MINLOC stay deterministic);
 *  DETERMINISTIC : root-sorted segmented reduction; FP SUM is the
 *                  canonical pairwise sum of the root's leaves in ascending
 *                  leaf index, added to the root (root on the left); FP
 *                  PROD the same tree with products, the root multiplied
 *                  last;
 *                  bit-identical for every launch configuration.
 * Roots with a single leaf never need atomics. */
typedef enum { SF_REDUCE_AUTO = 0, SF_REDUCE_ATOMIC = 1, SF_REDUCE_DETERMINISTIC = 2 } sf_reduce_mode;

/* Options of sf_setup (NULL = all defaults). */
typedef struct {
  int32_t reduce_mode;  /* sf_reduce_mode, default AUTO */
  int32_t use_patterns; /* 1 (default): detect contiguous / 3-D sub-block index patterns */
  int32_t analyze_only; /* 1: host analysis only, no device memory (for inspection) */
  int32_t partition;    /* Reduce / FetchAndOp through window-major scratch (units of at most
                           16 bytes, SFs with repeated roots): 0 auto (the deterministic
                           FetchAndOp from 2^16 leaves, the atomic Reduce from 2^19, the
                           deterministic Reduce from 2^19 when some root has more than 32
                           leaves and from 2^20 otherwise, the atomic FetchAndOp from 2^20),
                           1 always, 2 never.  Deterministic results are identical either way;
                           atomic results meet the same bar either way. */
  int32_t hot_path;     /* partitioned SFs whose leaf order is their segment order: 1 keeps the
                           leaves of the roots of highest degree (at least 2 per 8192 leaves on
                           average, at most 4096 roots) in leaf order -- per-tile partial results
                           combined per root -- for FetchAndOp and every Reduce but the
                           deterministic FP sum and MAXLOC; 0 (default) and 2 never (measured
                           no faster on a 16M-leaf Zipf SF).  Results are identical either way
                           (atomic ones meet the same bar). */
} sf_setup_opts;

/* Index pattern of one side of one segment (Section 5.2): index(t) for the
 * t-th leaf of the segment, t = i + dx*(j + dy*k), 0 <= i < dx, 0 <= j < dy,
 * 0 <= k < dz, is start + i + sy*j + sz*k (sy = X, sz = X*Y of the paper). */
typedef enum { SF_PATTERN_GENERIC = 0, SF_PATTERN_CONTIGUOUS = 1, SF_PATTERN_3D = 2 } sf_pattern_kind;
typedef struct {
  int32_t kind; /* sf_pattern_kind */
  int32_t start, dx, dy, dz, sy, sz;
} sf_pattern;

typedef struct {
  int64_t rank;    /* segment label */
  int64_t nleaves; /* leaves in the segment */
  sf_pattern root; /* pattern of the roots r_i of the segment's leaves */
  sf_pattern leaf; /* pattern of the leaf slots l_i */
} sf_segment_info;

typedef struct {
  int64_t nroots, nleaves;
  int64_t leafspace;      /* slots a leaf buffer must hold: max(ilocal)+1, or nleaves */
  int64_t nsegments;
  int64_t nroots_touched; /* roots of degree >= 1 */
  int64_t max_degree;
  int32_t has_dup_roots;  /* some root has degree >= 2 */
  int32_t reduce_mode;    /* current sf_reduce_mode */
  int64_t nhot;           /* roots aggregated in LDS by the atomic path */
  int64_t device_bytes;   /* device memory held by the plan */
  int64_t hot_roots;      /* roots whose leaves stay in leaf order on the partitioned path (hot_path) */
} sf_info;

/* Error codes. */
typedef enum {
  SF_OK = 0,
  SF_ERR_ARG = -1,         /* bad argument: size, index out of range, null pointer, misalignment */
  SF_ERR_DUP_LEAF = -2,    /* two leaves share a slot: stars must be disjoint (Section 3.1) */
  SF_ERR_NOT_SETUP = -3,   /* operation before sf_setup */
  SF_ERR_UNSUPPORTED = -4, /* unit/op combination or mode not provided */
  SF_ERR_HIP = -5,         /* HIP runtime or launch error */
  SF_ERR_OOM = -6,         /* device or host allocation failed */
  SF_ERR_MISMATCH = -7,    /* *_end without a matching *_begin with the same arguments */
  SF_ERR_BUSY = -8,        /* *_begin while the same operation on the same buffers is pending */
  SF_ERR_SCRATCH = -9      /* an allocation-free call needs more scratch than its fixed buffer holds */
} sf_error;

/* ------------------------------------------------------------- creation */

/* PetscSFCreate + PetscSFSetGraph (Section 3.1).
 *  nroots   : roots owned here, numbered 0..nroots-1.
 *  nleaves  : connected leaves.
 *  ilocal   : [nleaves] leaf slots (distinct, >= 0), or NULL for slots
 *             0..nleaves-1 (contiguous leaf space).
 *  iremote  : [nleaves] root address of each leaf; index in [0, nroots).
 *  localmode, remotemode: sf_copymode of the two arrays.
 *  out      : receives the new handle (NULL on error).
 * Errors: SF_ERR_ARG (negative sizes, index out of range, sizes >= 2^31,
 * NULL iremote with nleaves > 0), SF_ERR_DUP_LEAF, SF_ERR_UNSUPPORTED
 * (SF_OWN_POINTER), SF_ERR_OOM. */
int sf_create(int64_t nroots, int64_t nleaves, const int64_t *ilocal, int32_t localmode,
              const sf_node *iremote, int32_t remotemode, sf_t *out);

/* PetscSFSetUp (Section 3.1: internal structures, all optimisations, cost
 * amortised over many operations).  Groups leaves into segments by rank
 * (stable), detects per-segment index patterns (Section 5.2), detects
 * duplicate roots (Section 5.3), builds the root-sorted leaf lists of the
 * deterministic reduction and the hot-root table of the atomic one, and
 * uploads the index plan to the current device.  Synchronous.  Calling it
 * again rebuilds the plan with the new options. */
int sf_setup(sf_t sf, const sf_setup_opts *opts);

/* Change the reduce mode of a set-up SF (sf_reduce_mode). */
int sf_set_reduce_mode(sf_t sf, int32_t mode);

/* --------------------------------------------------------- communication */

/* SFBcast (Section 3.2, item 1): root -> leaves.  For every leaf i,
 * leafdata[l_i] = rootdata[r_i] (REPLACE) or op(leafdata[l_i], rootdata[r_i])
 * (SUM, MAX, MIN, PROD; MAXLOC, MINLOC on F64_I32).  Holes are not touched.
 *  rootdata: [nroots] units; leafdata: [leafspace] units. */
int sf_bcast_begin(sf_t sf, sf_unit unit, const void *rootdata, void *leafdata, int32_t op,
                   hipStream_t stream);
int sf_bcast_end(sf_t sf, sf_unit unit, const void *rootdata, void *leafdata, int32_t op,
                 hipStream_t stream);

/* SFReduce (Section 3.2, item 1, the reverse direction): leaves -> root, the root's
 * own value taking part (Section 4.1 adds B^T x back onto y).  Roots without
 * leaves are not touched.  REPLACE: the last leaf in leaf order wins
 * (deterministic mode; in atomic mode some leaf wins).  MAXLOC: larger
 * value wins, MINLOC: smaller value wins, equal values going to the smaller
 * index in both.  MAX/MIN (and the pairs' values) order -0 < +0.
 *  leafdata: [leafspace] units; rootdata: [nroots] units. */
int sf_reduce_begin(sf_t sf, sf_unit unit, const void *leafdata, void *rootdata, int32_t op,
                    hipStream_t stream);
int sf_reduce_end(sf_t sf, sf_unit unit, const void *leafdata, void *rootdata, int32_t op,
                  hipStream_t stream);

/* sf_reduce_begin for callers that cannot allocate memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, results and end call (sf_reduce_end) as sf_reduce_begin, but no
 * device or host memory is allocated and nothing is freed: the scratch the
 * kernels need comes from one fixed device buffer of SF_NOALLOC_SCRATCH_BYTES
 * (64 MiB) per device, which the library holds until the process ends.
 *  - A large SF whose partitioned path (window-major scratch copy of the
 *    leaves) needs more than the buffer runs the direct kernels instead:
 *    identical bits in DETERMINISTIC mode, the same tolerance in ATOMIC mode.
 *  - SF_ERR_SCRATCH when even the direct kernels need more (chunk levels of
 *    very large roots with wide units, or MAXLOC in ATOMIC mode with more
 *    than 8M touched roots x bs); nothing is enqueued then.
 *  - Every call on a device shares that device's buffer, which keeps the
 *    last call's contents (no kernel relies on it holding anything at the
 *    start).  Calls that overlap in time on one device -- on two streams, or
 *    from two threads -- race on it: order them on one stream.
 *  - SF_ERR_BUSY also when too many operations of this SF are pending. */
#define SF_NOALLOC_SCRATCH_BYTES (64u << 20)
int sf_reduce_begin_noalloc(sf_t sf, sf_unit unit, const void *leafdata, void *rootdata, int32_t op,
                            hipStream_t stream);

/* SFFetchAndOp (Section 3.2, item 2), op = SUM: every leaf i fetches the
 * current partial value of its root into leafupdate[l_i], then adds
 * leafdata[l_i] to it.  Deterministic mode (integer units): leaves are
 * applied in ascending leaf index, the result equals the sequential
 * definition bit for bit.  Atomic mode (any non-pair unit): each root's
 * leaves are applied in some order; the final root is the same, the fetched
 * values are the partial sums of that order.
 *  rootdata: [nroots] units, updated in place; leafdata, leafupdate:
 *  [leafspace] units (must not overlap). */
int sf_fetch_and_op_begin(sf_t sf, sf_unit unit, void *rootdata, const void *leafdata,
                          void *leafupdate, int32_t op, hipStream_t stream);
int sf_fetch_and_op_end(sf_t sf, sf_unit unit, void *rootdata, const void *leafdata,
                        void *leafupdate, int32_t op, hipStream_t stream);

/* ------------------------------------------------- composition (Section 3.3) */
/* New SFs from existing ones: host graph algebra on the graphs given to
 * sf_create; the results are created with their own copies of the graph and
 * are not set up.  Segment labels follow the leaves they come from. */

/* The graph of sf: ilocal[nleaves] (the slots, also when sf was created
 * with ilocal = NULL) and iremote[nleaves]; either may be NULL. */
int sf_get_graph(sf_t sf, int64_t *ilocal, sf_node *iremote);

/* PetscSFCreateEmbeddedRootSF: only the edges whose root is one of the n
 * selected roots remain; indices are not remapped (same nroots, same leaf
 * slots), so the new SF communicates on the original buffers.
 * Errors: SF_ERR_ARG (a root out of range), SF_ERR_OOM. */
int sf_create_embedded_root_sf(sf_t sf, int64_t n, const int64_t *selected_roots, sf_t *out);
/* PetscSFCreateEmbeddedLeafSF: only the edges whose leaf slot is one of the
 * n selected slots remain (a selected slot without a leaf selects nothing;
 * a negative one is SF_ERR_ARG); no remapping. */
int sf_create_embedded_leaf_sf(sf_t sf, int64_t n, const int64_t *selected_leaves, sf_t *out);

/* PetscSFCompose: a's leaf slots are b's roots (leafspace(a) <= nroots(b)).
 * ab has a's roots and b's leaves: b's leaf at slot l on root m becomes a
 * leaf of root r when a has a leaf at slot m on root r (b's leaves whose
 * root is no leaf of a are dropped), so Bcast on ab = Bcast on a, then on b. */
int sf_compose(sf_t a, sf_t b, sf_t *ab);
/* PetscSFComposeInverse: a's and b's leaves share one leaf space and every
 * root of b has at most one leaf (else SF_ERR_ARG).  ab has a's roots and
 * b's roots as its leaves: b's root m (whose leaf sits at slot l) becomes a
 * leaf of root r when a has a leaf at slot l on root r. */
int sf_compose_inverse(sf_t a, sf_t b, sf_t *ab);

/* ----------------------------------------------- multi-SF, Gather, Scatter */

/* The multi-SF of sf (PetscSFGetMultiSF, Section 3.2, item 2): every root r
 * of sf is split into deg(r) new roots, numbered from the exclusive prefix
 * sum of the degrees (so the new roots of r are consecutive, in the leaf
 * order of r's leaves), and leaf i of sf (same slot, same segment label) is
 * the only leaf of its new root.  Built on the current device the first time
 * it is asked for -- degrees by a Reduce SUM of ones, offsets by a scan, the
 * new roots by a FetchAndOp SUM in leaf order (roots starting at their
 * offsets, leaves adding 1) -- and then set up like any SF; synchronous.
 *  multi: receives a handle OWNED BY sf (do not destroy it); valid until sf
 *         is set up again or destroyed.  It has nleaves(sf) roots.
 * Errors: SF_ERR_NOT_SETUP, SF_ERR_ARG (another device current), SF_ERR_OOM,
 * SF_ERR_HIP. */
int sf_get_multi_sf(sf_t sf, sf_t *multi);

/* SFGather (PetscSFGatherBegin/End, Section 3.2, item 2): every leaf's unit
 * is copied to its new root in the multi-SF: multirootdata[m_i] =
 * leafdata[l_i], so multirootdata holds, root by root, each root's leaf
 * units in leaf order.  Builds the multi-SF on first use (synchronously).
 *  leafdata: [leafspace] units; multirootdata: [nleaves] units (any unit,
 *  whole units are copied). */
int sf_gather_begin(sf_t sf, sf_unit unit, const void *leafdata, void *multirootdata, hipStream_t stream);
int sf_gather_end(sf_t sf, sf_unit unit, const void *leafdata, void *multirootdata, hipStream_t stream);

/* SFScatter (PetscSFScatterBegin/End): the reverse of Gather,
 * leafdata[l_i] = multirootdata[m_i]; holes are not touched. */
int sf_scatter_begin(sf_t sf, sf_unit unit, const void *multirootdata, void *leafdata, hipStream_t stream);
int sf_scatter_end(sf_t sf, sf_unit unit, const void *multirootdata, void *leafdata, hipStream_t stream);

/* ------------------------------------------- sparse products (Section 4.1) */

/* A row-distributed sparse matrix is split on each rank into a diagonal
 * block A (columns of the rank's own vector entries) and an off-diagonal
 * block B (columns of the ghost vector lvec), both in CSR with reduced local
 * column indices; the ghost SF has the n vector entries as roots and lvec's
 * m entries as leaves (contiguous, ilocal = NULL). */
typedef struct sf_csr_s *sf_csr_t;

/* A CSR matrix of f64 values on the current device.  rowptr: [nrows + 1],
 * rowptr[0] = 0, non-decreasing; colidx, values: [rowptr[nrows]], colidx in
 * [0, ncols).  Host arrays, copied (also kept on the host for
 * sf_csr_transpose).  Errors: SF_ERR_ARG, SF_ERR_OOM, SF_ERR_HIP. */
int sf_csr_create(int64_t nrows, int64_t ncols, const int64_t *rowptr, const int32_t *colidx,
                  const double *values, sf_csr_t *out);
/* The transpose of a (a new matrix, built on the host and uploaded). */
int sf_csr_transpose(sf_csr_t a, sf_csr_t *out);
/* y = A x, or y += A x when accumulate != 0 (device pointers; x: [ncols],
 * y: [nrows]), on stream. */
int sf_csr_spmv(sf_csr_t a, const double *x, double *y, int32_t accumulate, hipStream_t stream);
int sf_csr_destroy(sf_csr_t *a);

/* y = M x for M = [A B] (Section 4.1): SFBcast REPLACE of x to lvec on sf
 * runs on comm_stream, overlapped with y = A x on stream; stream then waits
 * for the Bcast (an event) and computes y += B lvec.  A: n x n with n =
 * nroots(sf); B: n x leafspace(sf).  x: [n], lvec: [leafspace], y: [n],
 * device f64.  Enqueues only; results are visible in stream order on stream.
 * comm_stream must have the default priority. */
int sf_spmv(sf_t sf, sf_csr_t A, sf_csr_t B, const double *x, double *lvec, double *y, hipStream_t stream,
            hipStream_t comm_stream);
/* y = M^T x: y = A^T x, lvec = B^T x, then SFReduce SUM of lvec onto y, all
 * on stream.  At, Bt: sf_csr_transpose of A and B (At: n x n, Bt:
 * leafspace x n). */
int sf_spmv_transpose(sf_t sf, sf_csr_t At, sf_csr_t Bt, const double *x, double *lvec, double *y,
                      hipStream_t stream);

/* --------------------------------------------------------------- batches */

typedef enum { SF_KIND_BCAST = 0, SF_KIND_REDUCE = 1, SF_KIND_FETCH_AND_OP = 2 } sf_kind;

/* One operation of a batch: an SF (set up), a unit, a kind, an op and the
 * device buffers (roots, leaves; FetchAndOp also leafupdate, which must not
 * be leafdata; NULL for the other kinds). */
typedef struct {
  sf_t sf;
  sf_unit unit;
  int32_t kind; /* sf_kind */
  int32_t op;   /* REPLACE for Bcast; SUM for Reduce and FetchAndOp */
  void *rootdata;
  void *leafdata;
  void *leafupdate;
} sf_batch_item;

/* Batch many independent SF operations (uneven sizes, units and kinds) so
 * that they run in ONE kernel launch (Section 5.4: launch costs
 * that small kernels cannot hide).  The work table is built once here; the
 * buffers of the items are bound to the batch (the same pointers are used by
 * every launch).  The items' SFs must stay alive while the batch exists and
 * no two items may write the same buffer; an item whose SF is set up again
 * after this call makes every later call on the batch return
 * SF_ERR_NOT_SETUP (create a new batch).  Reduce items use atomics for roots
 * of several leaves unless their SF is in DETERMINISTIC mode (AUTO: roots of
 * more than 256 leaves take atomics).  FetchAndOp items (SUM) on integer
 * units run in leaf order -- bit-identical to sf_fetch_and_op -- unless
 * their SF is in ATOMIC mode; floating-point units use returning atomics.
 * Autotuning of the launch shape is sf_batch_autotune's, per batch (not an
 * option of sf_setup). */
int sf_batch_create(int32_t n, const sf_batch_item *items, sf_batch_t *out);

/* Run every item of the batch in one launch on stream. */
int sf_batch_launch(sf_batch_t batch, hipStream_t stream);

/* Run the items one kernel launch per item (the per-SF comparison). */
int sf_batch_launch_separate(sf_batch_t batch, hipStream_t stream);

/* Capture the batch's launch sequence (mode 0: the single batch
 * launch, mode 1: one launch per item) into a HIP graph on stream; later
 * sf_batch_graph_launch calls replay it.  Scratch memory the items need is
 * allocated before the capture.  sf_batch_set_config and sf_batch_autotune
 * drop the captured graph (capture again afterwards). */
int sf_batch_graph_capture(sf_batch_t batch, int32_t mode, hipStream_t stream);
int sf_batch_graph_launch(sf_batch_t batch, hipStream_t stream);

/* Time the candidate launch shapes (leaves per thread x tile size) of the
 * batch kernel on stream and keep the fastest.  cache_path (may be
 * NULL) names a text file of earlier choices keyed by the batch's shape: a
 * hit skips the timing, a miss appends the result.  The candidates are
 * bit-identical in every result that is deterministic.  Launches the batch
 * several times: the item buffers are overwritten. */
int sf_batch_autotune(sf_batch_t batch, const char *cache_path, hipStream_t stream);

/* Current launch shape (leaves per thread, tile leaves) and work tiles. */
int sf_batch_get_config(sf_batch_t batch, int32_t *lpt, int32_t *tile, int64_t *ntiles);
int sf_batch_set_config(sf_batch_t batch, int32_t lpt, int32_t tile);
int sf_batch_destroy(sf_batch_t *batch);

/* ----------------------------------------------------------- inspection */

int sf_get_info(sf_t sf, sf_info *info);
/* Segment s (0 <= s < nsegments) after sf_setup. */
int sf_get_segment(sf_t sf, int64_t s, sf_segment_info *seg);
const char *sf_error_string(int code);
/* The HIP error behind the last SF_ERR_HIP of the calling thread. */
int sf_last_hip_error(void);
/* Destroy the SF, free its device memory; *sf is set to NULL. */
int sf_destroy(sf_t *sf);

#ifdef __cplusplus
}
#endif
#endif /* SF_H */
