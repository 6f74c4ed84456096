// Internal declarations shared by the HIP kernels and the host runtime of
// libltl4c.  Not part of the public ABI (include/ltl4c.h is).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ltl4c {

constexpr int kMaxProps = 16;
constexpr int kMaxLevels = 4;
constexpr int kStates = 16;          // monitor states, at most (a map holds one byte per state)
constexpr int kRadixBits = 8;
constexpr int kRadixBitsWide = 9;        // digit of the passes of 512-thread tiles, when it saves a pass
constexpr int kHistWords = 4096;         // classify's histograms: n_pass << digit bits, at most
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;     // 4096 words per tile
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;     // 4096 words per tile
constexpr int kCountThreads = 256;
constexpr int kCountWindow = 64;     // nodes kept in LDS per counting tile
constexpr uint32_t kSpinLimit = 1u << 22;   // bounded waits in decoupled look-back
constexpr uint32_t kMaxChunks = 4096;        // chunks in one stream-group push

// Error bits raised on the device and reported by ltl4c_wait():
//   kErrRange     an event key wider than its declared key_bits
//   kErrCapacity  more instances, nodes or bindings than the capacity
//   kErrSpin      a bounded look-back wait expired
//   kErrData      an internal consistency check failed (a verdict byte
//                 outside 0..5, a radix scatter destination past the kept
//                 events); such values are dropped, never written
enum : uint32_t { kErrRange = 1u, kErrCapacity = 2u, kErrSpin = 4u, kErrData = 8u };

// One property as the kernels see it (lives in device memory).
struct PropDev {
    uint8_t label[kStates];
    uint32_t bmap[16][4];            // class c -> map q -> delta(q, c), byte q of the 16 (identity for q >= n_states)
    uint32_t blabel[2];              // label of state q in bits 4(q mod 8).. of word q / 8
    uint32_t q0, n_states;
    uint32_t kind[kMaxLevels], op[kMaxLevels], num[kMaxLevels], den[kMaxLevels];
};

struct Plan {
    PropDev prop[kMaxProps];
    uint8_t class_of_type[256];
    uint8_t key_present[256];
};

// Look-back rows of one scan launch, per kind (aggregate / inclusive): the
// four instance / node counts and up to 16 map dwords.  The rows of a launch
// occupy 2 * kScanRows * tiles 32-bit words.
constexpr int kScanRows = 20;
constexpr int kScanGroupProps = 8;      // properties of one scan launch, at most

struct ClassifyArgs {
    const uint8_t* records;
    uint64_t n;
    uint32_t record_bytes;
    uint32_t type_dw, type_shift, type_mask;
    uint32_t n_keys;
    uint32_t key_dw[kMaxLevels], key_shift[kMaxLevels], key_mask[kMaxLevels], key_bits[kMaxLevels];
    uint32_t need_mask;              // key_present bits every event must carry
    uint32_t n_preds;                // data predicates: class += (holding predicates' bits) << pred_class_shift
    uint32_t pred_class_shift;
    uint32_t pred_dw[3], pred_shift[3], pred_mask[3], pred_op[3], pred_val[3];
    uint32_t check_type_range;       // the type field can exceed 255
    uint32_t cbits;
    uint32_t ibits;                  // trace index bits between the class and the key (0: none)
    uint32_t excl_shift;             // bit set in the word of an excluded event
    uint32_t n_pass;                 // radix passes whose histograms are built here
    uint32_t digit_bits;             // radix digit width (8 or 9)
    uint32_t sort_shift;             // lowest sorted bit
    const Plan* plan;
    uint64_t* words;
    uint32_t* hist;                  // [n_pass][1 << digit_bits]
    uint32_t* n_valid;               // non-null: count of events kept; excluded events enter no histogram
    uint32_t* err;
    // stream groups: event i belongs to the chunk c with
    // chunk_off[c] <= i < chunk_off[c+1]; its stream id goes above the keys
    const uint32_t* chunk_off;       // [n_chunks + 1], or nullptr
    const uint32_t* chunk_stream;    // [n_chunks]
    const uint64_t* chunk_ptr;       // [n_chunks] device address of each chunk, or nullptr
    uint32_t n_chunks;
    uint32_t stream_shift;
    uint32_t vec_ok;                 // every record address is 16-byte aligned (16-byte records)
    // parent events: a type whose key_present bits (within need_mask) equal
    // parent_mask carries every key but the innermost; such an event gets
    // the innermost key 0 and the kind bit at stream_shift, and is counted in
    // n_par.  parent_mask > need_mask: no parent events.
    uint32_t parent_mask;
    uint32_t* n_par;
    // ranked keys: key m of event i is rank[m][i] instead of its record field
    const uint32_t* rank[kMaxLevels];
};

struct SortPassArgs {
    const uint64_t* in;
    uint64_t* out;
    uint32_t n;                      // words in `in` (an upper bound when n_valid is set)
    uint32_t shift;                  // lowest bit of this pass's digit
    uint32_t nbits;                  // digit width (<= the kernel's digit bits)
    const uint32_t* hist;            // this pass's global histogram [buckets]
    uint32_t* status;                // [tiles][buckets] look-back words
    uint32_t* ticket;
    const uint32_t* n_valid;         // non-null: words kept by the first pass (device)
    uint32_t drop_excl;              // first pass: words with bit excl_shift set are dropped
    uint32_t excl_shift;
    uint32_t* err;
};

struct ScanArgs {
    const uint64_t* words;
    uint32_t n;
    const uint32_t* n_dev;               // non-null: the word count lives on the device (n bounds it)
    uint32_t cbits;
    uint32_t n_levels;
    uint32_t prefix_shift[kMaxLevels];   // word >> prefix_shift[m] = packed keys 0..m-1 (m>=1)
    uint32_t valid_shift;                // word >> valid_shift != 0 means excluded
    uint32_t n_props;                    // properties of this launch: plan->prop[prop_idx[0 ..]]
    uint8_t prop_idx[kScanGroupProps];
    uint32_t n_props_all;                // properties of the evaluation (node counts to zero)
    uint32_t structure;                  // this launch writes the numbering, parents, keys and sizes
    const Plan* plan;
    uint8_t* inst_verdict;               // [n_props_all][inst_stride]
    uint64_t inst_stride;
    uint64_t inst_limit;                 // instances with an id below this are written
    uint64_t* inst_keys;                 // optional [inst_limit]
    uint32_t* node_start[kMaxLevels];    // level m: first child of node j
    uint32_t* node_counts[kMaxLevels];   // level m: [p][node_stride][6], zeroed when node j is created
    uint64_t node_stride[kMaxLevels];
    uint32_t* inst_parent;               // optional [inst_limit]: level n_levels-1 node of each instance
    uint32_t* inst_conc;                 // optional [n_props_all][inst_stride]: first conclusive position (timeline)
    uint32_t* inst_start;                // with inst_conc: sorted position of every instance's first word
    uint8_t* event_verdict;              // optional [n_props_all][n_events]: verdict after every event, trace order
    uint64_t n_events;                   // row stride of event_verdict
    uint32_t class_mask;                 // class bits of a word (below the trace index, if any)
    uint32_t index_shift, index_mask;    // trace index of a word: (word >> index_shift) & index_mask
    uint64_t* node_keys[kMaxLevels];     // optional
    uint64_t node_limit[kMaxLevels];     // nodes with an id below this are written
    uint32_t* status;                    // look-back rows [2 * kScanRows][tiles], zeroed before the launch
    uint32_t emit_state;                 // write final states instead of verdicts
    uint32_t max_states;                 // largest monitor among the properties of this launch
    uint32_t* ticket;
    uint64_t* sizes;                     // [1 + n_levels] written by the last tile
    uint32_t* sizes32;                   // same, 32-bit, for the counting kernels
    uint32_t* err;
    // the split map scan (reduce, spine, down sweep; mapscan.hip)
    uint8_t* desc;                       // [n] per word: class | head << 4 | level-m heads << (4 + m)
    uint32_t read_desc;                  // 1: read the descriptors instead of the words
    uint32_t* agg;                       // [tiles][kMsRec] tile aggregates: 4 head counts, map dwords
    uint32_t* prefix;                    // [tiles][kMsRec] exclusive prefixes of the aggregates
    uint32_t* chunk_agg;                 // [chunks][kMsRec] spine of many tiles: chunk compositions
    uint32_t* chunk_pre;                 // [chunks][kMsRec] and their exclusive prefixes
    uint32_t spine_chunk;                // tiles per spine chunk
    uint32_t* trec;                      // [kMsThreadRec][tiles * kMsThreads] per thread: its exclusive
                                         // prefix within the tile (two packed head-count words, map dwords)
    uint32_t tiles;
};
// the split map scan: tiles of 256 threads x 16 or 32 words, and their records
constexpr int kMsThreads = 256;
constexpr int kMsSpineThreads = 1024;  // the spine block; a spine chunk holds at least this many tiles
constexpr int kMsTileMin = kMsThreads * 16;   // workspace arrays are sized for the smaller tile
constexpr int kMsRec = 4 + 16;
constexpr int kMsThreadRec = 2 + 16;

constexpr uint32_t kNever = 0xFFFFFFFFu;     // timeline: the instance never became conclusive

struct InstConclusiveArgs {
    uint32_t* inst_conc;                 // [n_props][inst_stride], positions in, word counts out
    const uint32_t* inst_start;          // [inst_limit]
    const uint32_t* n_inst;              // device count of instances
    uint64_t inst_limit, inst_stride;
    uint32_t n_props;
};

struct FinalizeArgs {
    uint32_t n_props;
    const Plan* plan;
    const uint32_t* root_counts;         // [p][6]
    uint8_t* root_verdict;
    uint64_t* root_counts_out;
    const uint64_t* sizes_ws;            // [n_levels] from the scan
    uint64_t* sizes_out;                 // [1 + n_levels]
    uint32_t n_levels;
};

struct CountArgs {
    uint32_t level;                      // m: the parents' level (0 = root)
    uint32_t n_levels;
    uint32_t n_props;
    const Plan* plan;
    // children
    const uint32_t* n_children;          // device count of children
    const uint32_t* child_parent;        // optional: parent node of every child (else found in node_start)
    uint32_t items;                      // children per thread and tile: 16 (leaves) or 2
    uint32_t* done;                      // non-null at the root: the last block to finish runs `fin`
    FinalizeArgs fin;
    uint64_t child_limit;                // children beyond this were not recorded
    const uint8_t* child_verdict;        // level m+1 == n_levels: instance verdicts [p][child_stride]
    const uint32_t* child_counts;        // otherwise: counts of level m+1 [p][child_stride][6]
    uint64_t child_stride;
    uint8_t* child_verdict_out;          // optional: verdicts of level m+1 nodes [p][child_stride]
    // parents
    const uint32_t* node_start;          // level m >= 1: CSR first child per node
    const uint32_t* n_nodes;             // device count of level-m nodes (m >= 1)
    uint64_t node_limit;                 // nodes beyond this were not recorded
    uint32_t* counts;                    // [p][stride][6]
    uint64_t stride;
    uint32_t* err;
};

struct ZeroArgs {
    uint32_t* ptr;
    const uint32_t* n_dev;               // if non-null: words = min(*n_dev, limit) * mult
    uint64_t mult;
    uint64_t n_words;                    // used when n_dev is null
    uint64_t limit;
};


// Online monitoring: the resident monitor tree of a stream group.
// Bindings and quantifier nodes live in open-addressing hash tables keyed by
// the packed (stream, key...) prefix; a node's id is its slot.
constexpr uint64_t kEmptyKey = ~0ull;
// A slot of a closed stream: skipped by lookups, reusable by inserts.  Real
// keys stay below 2^63, so neither marker is ever a key.
constexpr uint64_t kDeadKey = ~0ull - 1ull;
constexpr uint8_t kNoVerdict = 0xFF;     // node not yet counted in its parent

struct GroupState {
    uint32_t n_props, n_levels;
    uint32_t vbase[kMaxProps];           // first virtual property of property p
    const Plan* plan;                    // real properties (labels, q0, quantifiers)
    uint32_t level_shift[kMaxLevels];    // key >> level_shift[m] = (stream, keys 0..m-1), m >= 1
    uint32_t stream_shift;               // key >> stream_shift = stream
    uint32_t max_streams;
    uint32_t* stream_max;                // [max_streams]: bindings a stream may hold
    // bindings
    uint64_t* bslot;                     // [bcap][2]: key, then parent | states of properties 0..3 << 32
    uint64_t bmask;
    uint8_t* bstate;                     // [P - 4][bcap]: states of properties 4..
    uint32_t* stream_bindings;           // [max_streams]
    // quantifier nodes of levels 1..n_levels-1
    uint64_t* nkeys[kMaxLevels];         // [ncap]
    uint64_t nmask;
    uint32_t* ncounts[kMaxLevels];       // [P][ncap][6]
    uint8_t* nverdict[kMaxLevels];       // [P][ncap]
    uint32_t* nparent[kMaxLevels];       // [ncap]
    uint32_t* ndirty[kMaxLevels];        // [ncap]
    uint32_t* nlist[kMaxLevels];         // [ncap]
    // stream roots
    uint32_t* rcounts;                   // [S][P][6]
    uint8_t* rverdict;                   // [S][P]
    uint32_t* rdirty;                    // [S]
    uint32_t* rlist;                     // [S]
    uint32_t* list_cnt;                  // [kMaxLevels]: dirty-list lengths (index 0 = roots)
    uint32_t* err;
};

struct GroupUpdateArgs {
    GroupState g;
    const uint32_t* n_seg;               // segments (instances) of this push
    const uint64_t* seg_key;             // [n_seg] packed (stream, keys)
    const uint8_t* seg_state;            // [V][seg_stride] final state per start state
    uint64_t seg_stride;
};

// Per-trace results of a batch: trace t's root is the level-1 node whose key
// is t (traces without events get Def. 7 on empty counts).
struct BatchOutArgs {
    uint32_t n_props, n_traces;
    const Plan* plan;
    const uint32_t* n_nodes;             // level-1 nodes
    const uint64_t* node_keys;           // [n_nodes] trace ids, increasing
    const uint32_t* node_counts;         // [P][stride][6]
    const uint8_t* node_verdict;         // [P][stride]
    uint64_t stride;
    uint8_t* verdict;                    // [n_traces][P]
    uint64_t* counts;                    // [n_traces][P][6]
};

// Parent events (an event with the keys of every level but the innermost
// joins every instance under its parent): after the radix sort the own events
// fill [0, n_own) of `words` and the parent events [n_own, n_own + n_par),
// the latter in (prefix, trace index) order.
constexpr int kPeThreads = 256;
constexpr int kPeItems = 16;
constexpr int kPeTile = kPeThreads * kPeItems;
constexpr int kPeSpineThreads = 1024;
constexpr int kPeShortGap = 8;          // gaps up to this many parent entries skip the segment tree
constexpr int kPeShortRun = 8;          // a parent's run up to this long is held in registers
constexpr int kPeSamples = 2048;        // sample table of the parent array (fits the word rows in LDS)
static_assert(kPeSamples <= kPeItems * kPeThreads, "samples share LDS with the staged words");
constexpr int kPeTreeLevelsPerLaunch = 8;
constexpr int kPeMaxTreeLevels = 33;
struct ParentArgs {
    const uint64_t* words;
    const uint32_t* n_kept;              // events kept by classify (own + parent)
    uint32_t* n_par;                     // parent events (classify counts them)
    uint32_t* n_own;                     // own events (k_pe_counts)
    uint32_t cbits;                      // class bits
    uint32_t class_mask;
    uint32_t ibits;                      // trace index bits above the class
    uint64_t index_mask;
    uint32_t key_shift;                  // word >> key_shift: the packed key (instance identity)
    uint32_t prefix_shift;               // (word >> prefix_shift) & prefix_mask: keys 0..n-2
    uint64_t prefix_mask;
    uint32_t n_props;
    const Plan* plan;
    uint4* tree;                         // segment tree levels 1..: [level][p][tree_cnt[level]]
    uint64_t tree_off[kPeMaxTreeLevels]; // in uint4 units
    uint64_t tree_cnt[kPeMaxTreeLevels];
    uint4* tile_agg;                     // [tiles][P]
    uint4* tile_prefix;                  // [tiles][P]
    uint4* trec;                         // [P][tiles * kPeThreads] each thread's run map
    uint64_t* samples;                   // [kPeSamples] keys of every stride-th parent entry
    uint32_t* tile_heads;                // [tiles]
    uint32_t* tile_head_prefix;          // [tiles]
    uint8_t* inst_verdict;               // [P][inst_stride]
    uint64_t inst_stride, inst_limit;
    uint32_t* err;
};

// Key ranking (composite keys wider than the sort word): per level, every
// event's value is replaced by its dense rank among the level's values.
constexpr int kRankThreads = 256;
constexpr int kRankItems = 16;
constexpr int kRankTile = kRankThreads * kRankItems;
constexpr int kRankSpineThreads = 1024;
struct RankArgs {
    const uint8_t* records;
    uint64_t n;
    uint32_t record_bytes;
    uint32_t type_dw, type_shift, type_mask;
    uint32_t has_key[8];                 // bit t: events of type t carry this level's key
    uint32_t level, key_dw, key_shift, key_mask;
    uint64_t* words;                     // prep: value << 32 | event index
    uint32_t* hist;                      // prep: [4][256] histograms of the value's bytes
    const uint64_t* sorted;              // the words after the radix passes over the value
    uint32_t* tile_cnt;                  // [tiles] distinct-value heads per tile
    uint32_t* tile_off;                  // [tiles] heads before each tile
    uint32_t* n_distinct;                // number of distinct values
    uint32_t* rank;                      // [n] rank of every event's value
    uint32_t* uniq;                      // [n] value of every rank
};
struct KeyValuesArgs {
    const uint64_t* packed;              // packed keys (or ranks) of instances or nodes
    const uint32_t* n_dev;               // how many (device)
    uint64_t limit;
    uint32_t n_fields;                   // values per key
    uint32_t shift[kMaxLevels];
    uint64_t mask[kMaxLevels];
    const uint32_t* uniq[kMaxLevels];    // per field: value of every rank, or null (the field is the value)
    uint64_t uniq_cap;                   // entries of each uniq array
    uint32_t* out;                       // [n][n_fields]
};

// Launchers (defined in kernels.hip, parent.hip and rank.hip).
hipError_t launch_zero(const ZeroArgs& a, uint32_t blocks, hipStream_t s);
hipError_t launch_classify(const ClassifyArgs& a, hipStream_t s);
hipError_t launch_sort_pass(const SortPassArgs& a, int variant, uint32_t digit_bits, hipStream_t s);
uint32_t sort_threads(int variant);   // threads per block of a sort variant
uint32_t sort_tile(int variant);      // words per radix tile of a sort variant
constexpr int kSortVariants = 7;
constexpr int kDefaultSortVariant = 1;     // 512 threads x 16 words
hipError_t launch_scan(const ScanArgs& a, int variant, hipStream_t s);
hipError_t launch_mapscan(const ScanArgs& a, int items, hipStream_t s);   // reduce, spine, down sweep
uint32_t scan_tile(int variant);      // words per scan tile of a scan variant
constexpr int kScanVariants = 6;
constexpr int kSplitScanVariant = 4;       // reduce / spine / down sweep (mapscan.hip), 16 words a thread
constexpr int kSplitScanVariant32 = 5;     // the same, 32 words a thread
constexpr int kDefaultScanVariant = 4;
hipError_t launch_count(const CountArgs& a, hipStream_t s);
hipError_t launch_finalize(const FinalizeArgs& a, hipStream_t s);
hipError_t launch_inst_conclusive(const InstConclusiveArgs& a, hipStream_t s);
hipError_t launch_fill_u8(uint8_t* p, uint8_t v, uint64_t n, hipStream_t s);
hipError_t launch_group_update(const GroupUpdateArgs& a, uint64_t max_seg, hipStream_t s);
hipError_t launch_group_level(const GroupState& g, uint32_t level, hipStream_t s);
hipError_t launch_group_roots(const GroupState& g, bool all, hipStream_t s);
hipError_t launch_group_purge(const GroupState& g, uint32_t stream, hipStream_t s);
hipError_t launch_group_nodes(const GroupState& g, uint32_t level, uint64_t* keys, uint32_t* counts, uint8_t* verdict,
                              uint64_t capacity, uint64_t* n_out, hipStream_t s);
hipError_t launch_set_u32(uint32_t* p, uint32_t v, hipStream_t s);
// Up to kPutWords 32-bit words carried by value in the launch itself: a
// device write of host data with no host buffer, copy or allocation.
constexpr uint32_t kPutWords = 448;
struct PutWords {
    uint32_t n;
    uint32_t w[kPutWords];
};
hipError_t launch_put_words(uint32_t* dst, const PutWords& a, hipStream_t s);
hipError_t launch_group_read(const GroupState& g, uint8_t* verdict, uint64_t* counts, uint64_t* bindings,
                             hipStream_t s);
hipError_t launch_fill_u64(uint64_t* p, uint64_t n, uint64_t v, hipStream_t s);
hipError_t launch_fill_u8(uint8_t* p, uint64_t n, uint8_t v, hipStream_t s);
hipError_t launch_batch_out(const BatchOutArgs& a, hipStream_t s);
hipError_t launch_parent_counts(const ParentArgs& a, hipStream_t s);
hipError_t launch_parent_samples(const ParentArgs& a, hipStream_t s);
hipError_t launch_parent_tree(const ParentArgs& a, uint32_t level0, uint32_t nlev, uint64_t max_nodes0, hipStream_t s);
hipError_t launch_parent_pass(const ParentArgs& a, bool down, uint64_t max_tiles, hipStream_t s);
hipError_t launch_parent_spine(const ParentArgs& a, hipStream_t s);
hipError_t launch_rank_prep(const RankArgs& a, hipStream_t s);
hipError_t launch_rank_scan(const RankArgs& a, hipStream_t s);
hipError_t launch_key_values(const KeyValuesArgs& a, uint64_t max_n, hipStream_t s);

}  // namespace ltl4c
