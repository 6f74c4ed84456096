/*
 * ltl4c.h -- C ABI of the MI355X LTL4-C trace-monitoring library.
 *
 * The library evaluates LTL4-C properties phi = Q_0 ... Q_{n-1} psi
 * (Section 2.4, Eq. 3-4 of arXiv 1411.2239) on an event trace that already
 * resides in device memory.  Its inputs follow the input line of Algorithm 1:
 * an LTL4 monitor of psi (Def. 6, as a transition table), the trace u, the
 * quantifier string Q and the key vector K used to extract the values of the
 * quantified variables (Section 4.1).  Its outputs are the truth value of the
 * property (the root of the monitor tree, Section 3.4) and, on request, the
 * verdict of every submonitor: every LTL4 instance and every quantifier node
 * with its 6-bin count vector (Def. 8).
 *
 * Conventions for every function:
 *  - the return value is a status code (LTL4C_OK = 0, negative on error);
 *    no C++ exception crosses the ABI;
 *  - argument validation is synchronous and happens before anything is
 *    enqueued; a call that returns an error has enqueued no work;
 *  - pointers documented as "device" must point to memory of the context's
 *    device; pointers documented as "host" are read during the call only;
 *  - work is enqueued on the context's stream (ltl4c_set_stream); results in
 *    device memory are valid once that stream has been synchronised, and
 *    ltl4c_wait() both synchronises and reports errors detected on the
 *    device (a key wider than declared, a capacity overflow);
 *  - a context is not thread-safe: one host thread drives it at a time.
 */
#ifndef LTL4C_H
#define LTL4C_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define LTL4C_OK            0
#define LTL4C_EINVAL       -1  /* malformed argument (table, quantifier, layout, pointer) */
#define LTL4C_ENOMEM       -2  /* device or host allocation failed; workspace too small */
#define LTL4C_ECAPACITY    -3  /* more nodes/bindings than the capacity given */
#define LTL4C_EDEVICE      -4  /* a HIP call failed; ltl4c_last_error() has its text */
#define LTL4C_EADMIT       -5  /* a stream could not be admitted within the memory budget */
#define LTL4C_ESEQ         -6  /* call on a closed stream or out of sequence */
#define LTL4C_EUNSUPPORTED -7  /* beyond the library's limits (see below) */
#define LTL4C_ERANGE       -8  /* an event carried a key wider than its declared width */

/* ---- truth values: B6 in lattice order F < Fc < Fp < Tp < Tc < T
 *      (Section 2.3); LTL4 verdicts (Def. 5) use F, Fp, Tp, T -------------- */
enum { LTL4C_BOT = 0, LTL4C_BOT_C = 1, LTL4C_BOT_P = 2,
       LTL4C_TOP_P = 3, LTL4C_TOP_C = 4, LTL4C_TOP = 5 };

/* ---- quantifiers (Def. 3, Eq. 4): A = percentage, E = instance count ---- */
enum { LTL4C_Q_PERCENT = 0, LTL4C_Q_COUNT = 1 };
enum { LTL4C_LT = 0, LTL4C_LE = 1, LTL4C_GT = 2, LTL4C_GE = 3, LTL4C_EQ = 4 };

/* Limits. */
#define LTL4C_MAX_STATES   16  /* states of one monitor (4-bit state codes) */
#define LTL4C_MAX_CLASSES  16  /* event classes (letters) of one layout */
#define LTL4C_MAX_LEVELS    4  /* quantifiers per property */
#define LTL4C_MAX_PROPS    16  /* properties evaluated in one call */
#define LTL4C_MAX_EVENTS   ((1ull << 30) - 1)   /* events per ltl4c_eval call */

typedef struct ltl4c_ctx ltl4c_ctx;

/*
 * Record layout and valuation extraction (epsilon(u_i, K), Section 4.1).
 * A record is record_bytes long (a multiple of 4, at most 256).  The event
 * type is an unsigned little-endian field of type_bytes (1, 2 or 4) at
 * type_offset; key m (the value of the quantified variable x_m) is an
 * unsigned field of key_bytes[m] (1, 2 or 4) at key_offset[m].  Every field
 * must be naturally aligned (offset a multiple of its size).
 *
 * class_of_type[t] is the letter (event class, < n_classes) of an event of
 * type t; the monitor tables are indexed by class.  key_present[t] has bit m
 * set when events of type t carry key m.  An event whose type is >= 256 or
 * lacks any of the n_keys keys belongs to no cluster (it is ignored, as the
 * set of value vectors of Eq. 5 only contains complete vectors).
 *
 * key_bits[m] (1..32) is the declared width of key m: every key value must be
 * below 2^key_bits[m].  A wider value is detected on the device and reported
 * as LTL4C_ERANGE by ltl4c_wait().  The composite binding key (key 0 in the
 * most significant bits) is packed into a 64-bit sort word with the class
 * bits (and, when asked for, the trace index and the parent-event kind bit)
 * and an exclusion bit.  When the declared widths do not fit 63 bits,
 * ltl4c_eval first replaces every key value by its dense rank among the
 * values of its level in the trace (ranks keep order and equality, so
 * clusters, tree and output order are unchanged) and packs ranks of
 * ceil(log2(distinct values)) bits; only if those still do not fit does it
 * report LTL4C_EUNSUPPORTED.  Ranking ends in one synchronous read of the
 * distinct-value counts, so graph capture and ltl4c_eval_noalloc refuse such
 * layouts (LTL4C_EUNSUPPORTED), as do batches and stream groups.  The packed
 * inst_keys and node_keys are then packed ranks; inst_key_values and
 * node_key_values give the values.
 *
 * Data predicates (propositions computed from a record's data, such as the
 * comparison of a session's average chunk size with a maximum in the paper's
 * cloud-storage case study, Section 5): predicate i holds for an event when
 * its field (an unsigned little-endian integer of pred[i].bytes = 1, 2 or 4
 * bytes at pred[i].offset, naturally aligned) compared by pred[i].op with
 * pred[i].value is true.  The event's class is then
 *   class_of_type[type] + (sum over holding predicates i of 2^i) << pred_shift,
 * which must stay below n_classes for every type and predicate outcome
 * (checked by ltl4c_set_layout).  n_preds = 0 leaves the class as
 * class_of_type[type].
 *
 * Parent events (parent_events = 1; the proxy-cache case study of Section 5,
 * where per-video events such as a cache insertion bear on every request of
 * the video): an event whose type carries keys 0 .. n_keys-2 and not key
 * n_keys-1 (for n_keys = 1: a type with no key) is a parent event.  It joins
 * the cluster u^D of every instance D whose first n_keys-1 values equal its
 * own, at its place in trace order; it creates no instance and no quantifier
 * node (the value vectors of Eq. 5 are the complete ones).  Events lacking
 * any other set of keys stay excluded.  The trace index of every event then
 * rides in the sort word: key bits + 1 + ceil(log2 n) + class bits must not
 * exceed 62, else ltl4c_eval reports LTL4C_EUNSUPPORTED.  Parent events are
 * supported by ltl4c_eval (and its graph and no-allocation forms), not by
 * batches or stream groups, and not with the verdict timeline outputs.
 */
enum { LTL4C_CMP_LT = 0, LTL4C_CMP_LE = 1, LTL4C_CMP_GT = 2, LTL4C_CMP_GE = 3, LTL4C_CMP_EQ = 4, LTL4C_CMP_NE = 5 };

typedef struct {
    uint32_t offset;
    uint32_t bytes;                  /* 1, 2 or 4 */
    uint32_t op;                     /* LTL4C_CMP_* */
    uint32_t value;
} ltl4c_pred;

typedef struct {
    uint32_t record_bytes;
    uint32_t type_offset;
    uint32_t type_bytes;
    uint32_t n_keys;                 /* number of quantifier levels, 1..4 */
    uint32_t key_offset[4];
    uint32_t key_bytes[4];
    uint32_t key_bits[4];
    uint32_t n_classes;              /* 1..16 */
    uint8_t  class_of_type[256];
    uint8_t  key_present[256];
    uint32_t n_preds;                /* data predicates, 0..3 */
    uint32_t pred_shift;             /* class bit of predicate 0 */
    ltl4c_pred pred[3];
    uint32_t parent_events;          /* 0 or 1, see above */
} ltl4c_layout;

/*
 * An LTL4 monitor (Def. 6): the deterministic machine (Sigma, Q, q0, delta,
 * lambda) with [u |=4 psi] = lambda(delta(q0, u)).  delta is row-major
 * [n_states][n_classes] with entries < n_states; label[q] is lambda(q), one of
 * LTL4C_BOT, LTL4C_BOT_P, LTL4C_TOP_P, LTL4C_TOP.  Host memory, copied.
 */
typedef struct {
    uint32_t n_states;               /* 1..16 */
    uint32_t n_classes;              /* must equal the layout's n_classes */
    uint32_t q0;
    const uint8_t *delta;
    const uint8_t *label;
} ltl4c_monitor;

/*
 * One counting quantifier Q_m = <kind, op, constant> (Eq. 4).  For
 * LTL4C_Q_PERCENT the constant is the exact rational num/den in [0, 1]
 * (den > 0, num <= den); for LTL4C_Q_COUNT it is the integer num (den ignored).
 * The numerical constraint S of Eq. 6 is evaluated exactly: k*den ~ num*N.
 */
typedef struct {
    uint32_t kind;
    uint32_t op;
    uint32_t num;
    uint32_t den;
} ltl4c_quant;

/* A property: monitor id from ltl4c_add_monitor and Q_0 (outermost) .. Q_{n-1}. */
typedef struct {
    int32_t monitor;
    uint32_t n_levels;               /* must equal the layout's n_keys */
    ltl4c_quant q[4];
} ltl4c_property;

/*
 * Outputs of one evaluation, all in device memory of the context's device.
 * Instances and nodes are numbered in increasing order of their (packed)
 * value vectors.  Optional arrays may be NULL; each optional array has room
 * for `capacity` entries per property, and a run that needs more reports
 * LTL4C_ECAPACITY from ltl4c_wait() (nothing beyond capacity is written).
 *
 *   root_verdict [n_props]                  truth value of each property
 *   root_counts  [n_props * 6]              child-verdict counts of the root
 *   sizes        [1 + n_levels]             sizes[0] = number of instances
 *                                           (full value vectors); sizes[m] =
 *                                           number of nodes at level m
 *                                           (m = 1..n_levels-1); unused
 *                                           entries are 0
 *   inst_keys    [capacity]                 packed value vector of instance i
 *   inst_verdict [n_props * capacity]       LTL4 verdict of instance i
 *   node_keys[m] [capacity]                 packed prefix (keys 0..m-1) of node j
 *   node_counts[m] [n_props * capacity * 6] 6-bin counts v of node j (Def. 8)
 *   node_verdict[m] [n_props * capacity]    verdict of node j
 *   inst_conclusive [n_props * capacity]    verdict timeline of instance i:
 *                                           the number of its events (in
 *                                           trace order) after which its
 *                                           verdict is first conclusive (T or
 *                                           F, final by Def. 5); 0 when the
 *                                           empty prefix already is;
 *                                           LTL4C_NEVER when no prefix is.
 *                                           Needs inst_verdict, and monitors
 *                                           whose T and F states only lead to
 *                                           states of the same label
 *                                           (LTL4C_EINVAL otherwise).
 *   event_verdict [n_props * n_events]     per event, in trace order: the
 *                                           verdict of the event's instance
 *                                           on its prefix up to and with the
 *                                           event; LTL4C_NO_INSTANCE for an
 *                                           event that joins no cluster.
 *                                           Needs the trace index beside the
 *                                           key in the sort word: binding key
 *                                           + class bits + ceil(log2 n_events)
 *                                           must fit 63 bits (else
 *                                           LTL4C_EUNSUPPORTED).
 *   inst_key_values [capacity * n_keys]     the values x_0..x_{n-1} of
 *                                           instance i (32 bits each); needs
 *                                           inst_keys
 *   node_key_values[m] [capacity * m]       the values x_0..x_{m-1} of node
 *                                           j; needs node_keys[m]
 * (node_* index m runs over 1..n_levels-1; index 0 is unused.)
 */
#define LTL4C_NEVER 0xFFFFFFFFu
#define LTL4C_NO_INSTANCE 0xFFu
/* (inst_keys and inst_verdict are given together or not at all; so are the
 * three node_* arrays of a level.) */
typedef struct {
    uint8_t  *root_verdict;
    uint64_t *root_counts;
    uint64_t *sizes;
    uint64_t  capacity;
    uint64_t *inst_keys;
    uint8_t  *inst_verdict;
    uint64_t *node_keys[4];
    uint32_t *node_counts[4];
    uint8_t  *node_verdict[4];
    uint32_t *inst_conclusive;
    uint8_t  *event_verdict;
    uint32_t *inst_key_values;
    uint32_t *node_key_values[4];
} ltl4c_result;

/* ---- context ----------------------------------------------------------- */

/* Create a context on HIP device `device`.  Work goes to the null stream
 * until ltl4c_set_stream() names another.  *out receives the context. */
int32_t ltl4c_create(ltl4c_ctx **out, int32_t device);
int32_t ltl4c_destroy(ltl4c_ctx *ctx);
/* Use `hip_stream` (a hipStream_t, may be NULL for the null stream). */
int32_t ltl4c_set_stream(ltl4c_ctx *ctx, void *hip_stream);
/* Text of the last error recorded on this thread (never NULL). */
const char *ltl4c_last_error(void);
const char *ltl4c_status_str(int32_t status);

/* Set the record layout; resets the registered properties. */
int32_t ltl4c_set_layout(ltl4c_ctx *ctx, const ltl4c_layout *layout);
/* Register a monitor; *id receives its id. EINVAL: entries out of range. */
int32_t ltl4c_add_monitor(ltl4c_ctx *ctx, const ltl4c_monitor *m, int32_t *id);
/* Register a property; *id receives its id. EINVAL: bad op/kind/constant. */
int32_t ltl4c_add_property(ltl4c_ctx *ctx, const ltl4c_property *p, int32_t *id);

/* ---- offline evaluation (Algorithm 1: SortTrace, SpawnMonitors,
 *      Distribute, ApplyQuantifiers) -------------------------------------- */

/* Bytes of device workspace ltl4c_eval needs for n_events events and the
 * properties `props` (n_props of them). */
int32_t ltl4c_workspace_bytes(ltl4c_ctx *ctx, uint64_t n_events, const int32_t *props,
                              int32_t n_props, uint64_t *bytes);

/* Evaluate the properties `props` (host array of ids) on the trace
 * d_records (device, n_events records in trace order).  d_workspace is
 * caller-owned device memory of at least the queried size, 256-byte aligned;
 * it is clobbered.  Asynchronous on the context's stream. */
int32_t ltl4c_eval(ltl4c_ctx *ctx, const void *d_records, uint64_t n_events,
                   const int32_t *props, int32_t n_props,
                   void *d_workspace, uint64_t workspace_bytes,
                   const ltl4c_result *out);

/* ---- evaluation without allocation ----------------------------------------
 *
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * evaluation as ltl4c_eval (same outputs, same errors), with the workspace and
 * the property table in a fixed scratch array that the library holds on every
 * device it runs on, from load to process end (LTL4C_NOALLOC_SCRATCH_BYTES per
 * device).  The call allocates nothing (no device or pinned memory, no
 * events; the property table travels to the device inside kernel launches)
 * and enqueues kernels only.  A trace whose ltl4c_workspace_bytes() exceeds
 * the scratch (minus the 6 KiB property table) is refused with LTL4C_ENOMEM;
 * one 16-byte-record trace of the two-level user/request shape fits up to
 * about 2.8 million events.  All calls on one device share that device's
 * scratch: calls that overlap in time on one device (two streams, two host
 * threads) race and give wrong results; serialise them.  Profiling
 * (ltl4c_profile_enable) does not time these calls. */
#define LTL4C_NOALLOC_SCRATCH_BYTES (64ull << 20)
int32_t ltl4c_eval_noalloc(ltl4c_ctx *ctx, const void *d_records, uint64_t n_events,
                           const int32_t *props, int32_t n_props, const ltl4c_result *out);

/* ---- batches: many independent traces in one pass -------------------------
 *
 * Evaluate the properties on n_traces (1..4096) independent traces at once:
 * trace t is records [offsets[t], offsets[t+1]) of d_records (offsets is a
 * host array of n_traces + 1 entries, offsets[0] = 0).  The trace id becomes
 * the top of the sort key, so every kernel of ltl4c_eval runs once for the
 * whole batch.  Outputs (device): root_verdict[t * n_props + p] and
 * root_counts[(t * n_props + p) * 6 + b], the same values ltl4c_eval gives for
 * trace t alone.  Properties of a batch have at most 3 quantifiers. */
int32_t ltl4c_batch_workspace_bytes(ltl4c_ctx *ctx, uint64_t n_events, int32_t n_traces, const int32_t *props,
                                    int32_t n_props, uint64_t *bytes);
int32_t ltl4c_eval_batch(ltl4c_ctx *ctx, const void *d_records, const uint64_t *offsets, int32_t n_traces,
                         const int32_t *props, int32_t n_props, void *d_workspace, uint64_t workspace_bytes,
                         uint8_t *d_root_verdict, uint64_t *d_root_counts);

/* Synchronise the context's stream and report device-detected errors of the
 * work enqueued since the previous ltl4c_wait (LTL4C_ERANGE, ECAPACITY). */
int32_t ltl4c_wait(ltl4c_ctx *ctx);

/* ---- online monitoring: stream groups ----------------------------------
 *
 * Online mode of Section 4: the monitor tree persists across invocations and
 * every new piece of trace updates it incrementally (the truth value evolves
 * with the trace).  A stream group keeps the trees of up to max_streams
 * independent traces ("streams") resident in device memory, all monitored for
 * the same properties with the context's layout.  Per binding (full value
 * vector) it keeps the monitor state of every property (the LTL4 submonitor of
 * Section 3.1); per quantifier node its 6-bin count vector and verdict
 * (Def. 8); per stream the root verdict.  Instantiation on first occurrence
 * (Section 3.3) is a device hash-table insert; after each push only the
 * touched nodes are re-valued, level by level up to the roots.
 *
 * Limits: the monitors of the group's properties have at most 16 states in
 * total; a push carries at most 4096 chunks and max_batch events; the stream
 * id, the keys and the class bits fit in 63 bits.  The library allocates the
 * group's device memory itself, within the context's memory budget. */

/* Cap on the device memory the context's stream groups may hold (default:
 * unlimited).  A group (or its host-ingestion staging) that would exceed it
 * is refused with LTL4C_EADMIT. */
int32_t ltl4c_set_memory_budget(ltl4c_ctx *ctx, uint64_t bytes);

/* Device bytes a group with these limits would take. */
int32_t ltl4c_group_bytes(ltl4c_ctx *ctx, const int32_t *props, int32_t n_props, uint32_t max_streams,
                          uint32_t max_bindings, uint64_t max_batch, uint64_t *bytes);

/* Open a group: max_bindings bounds the bindings of one stream, max_batch the
 * events of one push.  *group receives its id.  Synchronous. */
int32_t ltl4c_group_open(ltl4c_ctx *ctx, const int32_t *props, int32_t n_props, uint32_t max_streams,
                         uint32_t max_bindings, uint64_t max_batch, int32_t *group);
int32_t ltl4c_group_close(ltl4c_ctx *ctx, int32_t group);

/* Append n_chunks chunks: chunk i is records [offsets[i], offsets[i+1]) of
 * d_records (device, trace order) and continues stream streams[i].
 * offsets[0] = 0; chunks of one stream appear in arrival order.  offsets and
 * streams are host arrays read during the call.  Asynchronous on the
 * context's stream; the records must stay valid until it has run.
 * Bindings beyond max_bindings or a full table give LTL4C_ECAPACITY from
 * ltl4c_wait(). */
int32_t ltl4c_group_push(ltl4c_ctx *ctx, int32_t group, const void *d_records, const uint64_t *offsets,
                         const uint32_t *streams, int32_t n_chunks);

/* The same with every chunk in its own device buffer: chunk i is sizes[i]
 * records at d_chunks[i] (host arrays of n_chunks entries). */
int32_t ltl4c_group_push_chunks(ltl4c_ctx *ctx, int32_t group, const void *const *d_chunks, const uint64_t *sizes,
                                const uint32_t *streams, int32_t n_chunks);

/* Current truth values (device outputs): root_verdict[s * n_props + p],
 * root_counts[(s * n_props + p) * 6 + b], bindings[s] (may be NULL). */
int32_t ltl4c_group_read(ltl4c_ctx *ctx, int32_t group, uint8_t *d_root_verdict, uint64_t *d_root_counts,
                         uint64_t *d_bindings);

/* The quantifier nodes of level `level` (1..n_levels-1) of every stream, in
 * no particular order (device outputs, room for `capacity` nodes):
 * keys[j] = the node's packed prefix with the stream id above key 0 (the
 * stream id takes ceil(log2 max_streams) bits, or 1, and each key m its
 * key_bits[m]); counts[(p * capacity + j) * 6 + b] its 6-bin count vector
 * (Def. 8) and verdict[p * capacity + j] its verdict for property p; *d_n
 * (a device uint64) the number of nodes.  More nodes than capacity report
 * LTL4C_ECAPACITY from ltl4c_wait(). */
int32_t ltl4c_group_read_nodes(ltl4c_ctx *ctx, int32_t group, uint32_t level, uint64_t *d_keys, uint32_t *d_counts,
                               uint8_t *d_verdict, uint64_t capacity, uint64_t *d_n);

/* ---- streams of a group: admission, sequence numbers, host ingestion ----
 *
 * A group opened by ltl4c_group_open admits all its max_streams streams at
 * once, each with room for max_bindings bindings.  A group opened by
 * ltl4c_group_open_pool is a pool of pool_bindings binding slots (its hash
 * tables and node tables are sized for them, and charged to the memory
 * budget when it opens) with no stream admitted: ltl4c_stream_open admits one
 * stream with its own binding limit when the pool still has room for it
 * (LTL4C_EADMIT otherwise), and ltl4c_stream_close frees its slots and its
 * reservation.  Pushes to a stream that is not open fail with LTL4C_ESEQ.
 *
 * Every stream counts its chunks: ltl4c_group_push_seq takes each chunk's
 * sequence number and refuses the whole push (LTL4C_ESEQ, nothing enqueued)
 * unless every chunk carries its stream's next number, so a repeated chunk
 * or a lost one is caught before it reaches the monitor tree.  The other
 * push calls number their chunks implicitly.  ltl4c_stream_poll reports,
 * without blocking, the next number the stream expects and the number of
 * chunks whose verdict updates have completed on the device. */
int32_t ltl4c_group_open_pool(ltl4c_ctx *ctx, const int32_t *props, int32_t n_props, uint32_t max_streams,
                              uint64_t pool_bindings, uint64_t max_batch, int32_t *group);
/* Admit stream `stream` (< max_streams) with at most max_bindings bindings;
 * its first chunk will carry sequence number first_seq.  LTL4C_ESEQ if the
 * stream is already open.  Enqueued on the context's stream. */
int32_t ltl4c_stream_open(ltl4c_ctx *ctx, int32_t group, uint32_t stream, uint32_t max_bindings, uint64_t first_seq);
/* Close the stream: its bindings, nodes, counts and root are cleared (the
 * slots are reused by later inserts) and its reservation returns to the
 * pool.  Enqueued on the context's stream, after the pushes before it. */
int32_t ltl4c_stream_close(ltl4c_ctx *ctx, int32_t group, uint32_t stream);
/* *next_seq: the sequence number the stream's next chunk must carry;
 * *done_seq: every chunk numbered below it has been applied on the device
 * (its verdicts are visible to ltl4c_group_read).  Either may be NULL. */
int32_t ltl4c_stream_poll(ltl4c_ctx *ctx, int32_t group, uint32_t stream, uint64_t *next_seq, uint64_t *done_seq);
/* Open streams without a push for at least idle_ns nanoseconds (host steady
 * clock): up to `capacity` ids into streams[], their number in *n_stalled. */
int32_t ltl4c_group_stalled(ltl4c_ctx *ctx, int32_t group, uint64_t idle_ns, uint32_t *streams, uint32_t capacity,
                            uint32_t *n_stalled);
/* Push n_chunks chunks with sequence numbers: chunk i is sizes[i] records at
 * chunks[i], continuing stream streams[i] with number seqs[i] (host arrays).
 * is_device = 1: chunks[i] are device pointers (they must stay valid until
 * the push has run).  is_device = 0: chunks[i] are pinned host memory
 * (hipHostMalloc; pageable memory gives LTL4C_EINVAL); the library copies
 * them with the copy engine into one of two device staging buffers of
 * max_batch records (allocated at the first such push, within the memory
 * budget) on a copy stream of its own, so the copy of one push overlaps the
 * kernels of the previous one; the host memory must stay valid until
 * ltl4c_stream_poll reports the chunks done. */
int32_t ltl4c_group_push_seq(ltl4c_ctx *ctx, int32_t group, const void *const *chunks, const uint64_t *sizes,
                             const uint32_t *streams, const uint64_t *seqs, int32_t n_chunks, int32_t is_device);

/* Checkpoint / resume: copy the group's resident state to host memory
 * (*bytes is its size; host == NULL only queries it) and back.  Both
 * synchronise the context's stream.  The streams' admission and sequence
 * numbers are host state of the open group and are not part of it. */
int32_t ltl4c_group_snapshot(ltl4c_ctx *ctx, int32_t group, void *host, uint64_t *bytes);
int32_t ltl4c_group_restore(ltl4c_ctx *ctx, int32_t group, const void *host, uint64_t bytes);

/* ---- tuning ------------------------------------------------------------- */

/* Kernel schedule options (set before ltl4c_workspace_bytes, which depends
 * on them).  LTL4C_OPT_SORT_TILE selects the radix-pass tile shape:
 * 0 = 256 threads x 16 words, 1 = 512 x 16 (default), 2 = 256 x 24,
 * 3 = 256 x 8, 4 = 512 x 8, 5 = 512 x 12, 6 = 1024 x 16.  The shapes of 512
 * and more threads sort 9-bit digits when that takes fewer passes than 8-bit
 * ones. */
enum { LTL4C_OPT_SORT_TILE = 0, LTL4C_OPT_SCAN_TILE = 1 };
/* LTL4C_OPT_SCAN_TILE: 4 (default) = the split map scan: per tile of 4096
 * words (256 threads x 16) a reduce launch, one spine launch over the tiles,
 * a down-sweep launch, no look-back; 5 = the same with 8192-word tiles
 * (256 x 32).  0..3 = the single-pass look-back map scan with tiles
 * of 0 = 256 threads x 16 words, 1 = 512 x 16, 2 = 1024 x 16, or 3 = per
 * launch: 1024 x 16 when a launch's maps take at most 4 dwords per event (one
 * or two properties of at most 8 states, or one of at most 16), else
 * 512 x 16.
 * A value pins that tile: tuned schedules (below) no longer override it;
 * -1 returns the option to its default and unpins it. */
int32_t ltl4c_set_option(ltl4c_ctx *ctx, int32_t option, int64_t value);

/* ---- autotuned schedules ------------------------------------------------
 *
 * A schedule is the pair (radix-pass tile, map-scan tile) of the options
 * above.  The context keeps a table of tuned schedules keyed by a shape
 * class: single trace or batch of traces, packed key bits (with a batch's
 * trace id; they fix the radix passes), number of properties, whether some
 * monitor has more than 8 states, tree levels, and floor(log2(events)).
 * ltl4c_eval, ltl4c_eval_batch and the graph captures below run the tuned
 * schedule of their class (the entry of the nearest size within a factor of
 * 4) unless a tile is pinned; the workspace queries cover both the context's
 * own schedule and the tuned one, and a workspace too small for the tuned
 * one runs the context's own.  Results are identical under every schedule. */
typedef struct {
    int32_t sort_tile, scan_tile;     /* the chosen schedule */
    double tuned_us, default_us;      /* median time of one call under it and under the default */
    int32_t candidates;               /* schedules timed (those whose workspace fit) */
} ltl4c_tuned;

/* Workspace that every schedule of this call fits (the one to pass to
 * ltl4c_tune).  offsets == NULL: one trace of n_events; else a batch of
 * n_traces traces given by host offsets as in ltl4c_eval_batch. */
int32_t ltl4c_tune_workspace_bytes(ltl4c_ctx *ctx, uint64_t n_events, const uint64_t *offsets, int32_t n_traces,
                                   const int32_t *props, int32_t n_props, uint64_t *bytes);
/* Time the schedules on the caller's own data (device records, as for
 * ltl4c_eval / ltl4c_eval_batch) and record the fastest for its shape class,
 * replacing an entry of the same class and size.  Each candidate runs once to
 * warm up, then `reps` (1..1000) times; the median counts.  Coordinate
 * descent: every radix tile under the default scan tile, then every scan tile
 * under the best radix tile; a candidate must beat the best so far by 1 %.
 * Candidates whose workspace exceeds ws_bytes are skipped.  Synchronous:
 * returns when the timing is done; result may be NULL. */
int32_t ltl4c_tune(ltl4c_ctx *ctx, const void *d_records, uint64_t n_events, const uint64_t *offsets,
                   int32_t n_traces, const int32_t *props, int32_t n_props, void *d_workspace,
                   uint64_t workspace_bytes, int32_t reps, ltl4c_tuned *result);
/* Write the table as JSON, keyed by the device's architecture name (e.g.
 * "gfx950"); load such a file, ignoring it when it was tuned on another
 * architecture (*n_loaded = 0), replacing entries of the same class and
 * size; clear the table. */
int32_t ltl4c_schedule_save(ltl4c_ctx *ctx, const char *path);
int32_t ltl4c_schedule_load(ltl4c_ctx *ctx, const char *path, int32_t *n_loaded);
int32_t ltl4c_schedule_clear(ltl4c_ctx *ctx);

/* ---- graphs: captured kernel sequences -----------------------------------
 *
 * The same work as ltl4c_eval, ltl4c_eval_batch or ltl4c_group_push_chunks,
 * captured once into a HIP graph instead of run; ltl4c_graph_launch replays
 * it on the context's stream, one launch for the whole kernel sequence.
 * Arguments are validated as by the plain call, and the plan and the trace /
 * chunk table are copied to the device at capture (the graph owns its own
 * table), so a replay reads only device memory: the same record addresses,
 * outputs and workspace as at capture, whose contents may change between
 * replays (new records in the same buffers).  A group-push graph takes device
 * chunks only; every replay counts as one push of its chunks (sequence
 * numbers advance, ltl4c_stream_poll sees it) and needs its streams open.
 * Replays are ordered on the context's stream like any other call; a replay
 * and a plain call using one workspace must not overlap. */
int32_t ltl4c_graph_eval(ltl4c_ctx *ctx, const void *d_records, uint64_t n_events, const int32_t *props,
                         int32_t n_props, void *d_workspace, uint64_t workspace_bytes, const ltl4c_result *out,
                         int32_t *graph);
int32_t ltl4c_graph_eval_batch(ltl4c_ctx *ctx, const void *d_records, const uint64_t *offsets, int32_t n_traces,
                               const int32_t *props, int32_t n_props, void *d_workspace, uint64_t workspace_bytes,
                               uint8_t *d_root_verdicts, uint64_t *d_root_counts, int32_t *graph);
int32_t ltl4c_graph_group_push(ltl4c_ctx *ctx, int32_t group, const void *const *d_chunks, const uint64_t *sizes,
                               const uint32_t *streams, int32_t n_chunks, int32_t *graph);
int32_t ltl4c_graph_launch(ltl4c_ctx *ctx, int32_t graph);
/* Synchronises the context's stream, then frees the graph. */
int32_t ltl4c_graph_destroy(ltl4c_ctx *ctx, int32_t graph);

/* ---- profiling: per-kernel time of the enqueued work ------------------- */

/* When enabled, every kernel launch is bracketed by HIP events on the
 * context's stream and its duration accumulated per kernel name. */
int32_t ltl4c_profile_enable(ltl4c_ctx *ctx, int32_t on);
/* Synchronises, then reports kernel i (0-based): name (copied into name_buf
 * of name_len bytes), total milliseconds and launch count.  Returns
 * LTL4C_EINVAL when i is past the last kernel seen. */
int32_t ltl4c_profile_get(ltl4c_ctx *ctx, int32_t i, char *name_buf, int32_t name_len,
                          double *total_ms, uint64_t *launches);
int32_t ltl4c_profile_reset(ltl4c_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* LTL4C_H */
