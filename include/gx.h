/*
 * gx.h -- C ABI of an MI355X (gfx950) library for GPUexplore-style
 * explicit-state exploration and its bucketed find-or-put hash table,
 * after Cassee, Neele and Wijs, "On the Scalability of the GPUexplore
 * Explicit-State Model Checker" (GaM 2017, arXiv 1801.05857).
 *
 * Conventions for every call:
 *   - Every function returns a gx_status; GX_OK (0) on success, a negative
 *     code otherwise.  No exception crosses this boundary.
 *   - Argument errors return GX_EINVAL before any device work is queued, and
 *     leave every out-parameter untouched.
 *   - Pointers documented as "device" must point to memory of the GPU that was
 *     current when the table was created (e.g. a torch tensor's data_ptr()).
 *     Pointers documented as "host" are ordinary process memory.
 *   - A hip_stream argument is a hipStream_t passed as void*; NULL means the
 *     null stream.  Calls documented as "stream-ordered" only enqueue work.
 *   - Distinct tables are independent.  Concurrent gx_find_or_put calls on one
 *     table are linearisable per key.  Other calls on one table must not
 *     overlap with each other.
 */
#ifndef GX_H
#define GX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GX_OK = 0,
  GX_EINVAL = -1,     /* invalid argument, checked before any device work  */
  GX_ENOMEM = -2,     /* device or host allocation failed, or a buffer of  */
                      /* the call (frontier, deadlock list) was too small  */
  GX_ETABLEFULL = -3, /* a key exhausted every hash function (Sec. 4.1)    */
  GX_EDEVICE = -4,    /* a HIP runtime call failed                         */
  GX_EBUSY = -5,
  GX_ECANCELED = -6
} gx_status;

/* Per-key status byte written by gx_find_or_put. */
enum {
  GX_SEEN = 0,    /* the key was already stored                            */
  GX_NEW = 1,     /* this call stored the key                              */
  GX_FULL = 2,    /* every hash function led to a full bucket: not stored  */
  GX_INVALID = 3  /* a word of the key equals GX_EMPTY_WORD: not stored    */
};

/* Value of an unused table word.  No key word may take this value. */
#define GX_EMPTY_WORD 0xFFFFFFFFu

/* Opaque handle; owns its device storage. */
typedef struct gx_table gx_table;

typedef struct {
  uint64_t hash_seed;  /* seed of the hash-constant sets; 0 picks a fixed default */
  uint32_t max_hashes; /* H, hash functions tried before a key is FULL; 0 -> 8      */
  uint32_t subgroup;   /* lanes that probe one bucket: 4, 8, 16, 32 or 64
                          (lanes beyond bucket_words stay idle; a lane holds
                          at most 8 bucket words, so 4 needs bucket_words <=
                          32); 0 -> the larger of 8 and the smaller of
                          bucket_words and 64                                  */
  uint32_t keys_per_subgroup; /* keys a subgroup keeps in flight: 1, 2, 4 or 8,
                                 at most subgroup; 0 -> 1                        */
  uint32_t reserved;
} gx_table_opts;

/*
 * Create an empty table (Sec. 4.1: the storage is divided into buckets of
 * bucket_words 32-bit integers; vectors are stored inline, i.e. closed
 * hashing; Sec. 4.2: the bucket size is configurable).
 *
 *   words_per_state  w, 1..4.  Each key occupies a slot of S words, S = w for
 *                    w in {1,2,4} and S = 4 for w = 3 (the fourth word is 0).
 *   bucket_words     B, 4, 8, 16, 32 or 64.  A bucket holds B/S slots (a
 *                    bucket of 4 words holds one 4-word slot).
 *   capacity         number of keys the table must be able to hold; the table
 *                    gets ceil(capacity / (B/S)) buckets (at least 1).
 *   opts             nullable; see gx_table_opts.
 *   out              receives the handle.
 *
 * The storage is allocated with hipMalloc on the current device and cleared
 * (stream-ordered on the null stream, completed before return).
 * Errors: GX_EINVAL (bad w, B, subgroup, keys_per_subgroup or H, capacity 0),
 * GX_ENOMEM (allocation failed).
 */
gx_status gx_table_create(uint32_t words_per_state, uint32_t bucket_words, uint64_t capacity,
                          const gx_table_opts* opts, gx_table** out);

/* Free the table and its device storage.  NULL is accepted. */
gx_status gx_table_destroy(gx_table* table);

/* Reset every word to GX_EMPTY_WORD and the statistics to zero, with a fill
 * kernel on hip_stream (stream-ordered). */
gx_status gx_table_clear(gx_table* table, void* hip_stream);

/*
 * Find-or-put a batch of keys (Sec. 4.1 and 4.2): each key is looked up in the
 * bucket given by the first hash function; if it is not there it is stored in
 * the first free slot with a compare-and-swap; a bucket without a free slot
 * sends the key to the bucket of the next hash function; after H full buckets
 * the key is reported FULL and not stored.
 *
 *   keys     device, n * w uint32 words, row-major (key i = keys[i*w .. i*w+w)).
 *   n        number of keys; 0 is accepted and does nothing.
 *   status   device, n bytes; receives GX_NEW / GX_SEEN / GX_FULL / GX_INVALID
 *            per key.  When a key occurs several times among keys that were
 *            absent before the call, exactly one occurrence gets GX_NEW; which
 *            one is unspecified.
 *   n_new    device, nullable; when given, the number of GX_NEW keys is ADDED
 *            to *n_new (the caller zeroes it).
 *   hip_stream  stream-ordered; the call returns before the work completes.
 *
 * Errors: GX_EINVAL (null table/keys/status with n > 0), GX_EDEVICE (launch).
 */
gx_status gx_find_or_put(gx_table* table, const uint32_t* keys, uint64_t n, uint8_t* status,
                         uint64_t* n_new, void* hip_stream);

typedef struct {
  uint32_t words_per_state; /* w */
  uint32_t slot_words;      /* S */
  uint32_t bucket_words;    /* B */
  uint32_t subgroup;        /* lanes per bucket probe */
  uint32_t keys_per_subgroup;
  uint32_t max_hashes;      /* H */
  uint64_t n_buckets;
  uint64_t n_slots;         /* n_buckets * B / S */
  uint64_t hash_seed;
  uint64_t bytes;           /* device bytes of the bucket storage */
} gx_table_info;

/* Geometry of a table (host only, no device work). */
gx_status gx_table_get_info(const gx_table* table, gx_table_info* out);

typedef struct {
  uint64_t stored;      /* keys stored since the last clear (GX_NEW results)   */
  uint64_t lookups;     /* keys processed since the last clear                 */
  uint64_t probes;      /* bucket reads (first reads and re-reads)             */
  uint64_t full;        /* GX_FULL results                                     */
  uint64_t invalid;     /* GX_INVALID results                                  */
  uint32_t max_hash_index; /* largest hash index j used by a stored/found key */
  uint32_t reserved;
} gx_stats;

/* Statistics since the last clear.  Waits for all device work to finish. */
gx_status gx_table_stats(gx_table* table, gx_stats* out);

/*
 * Copy the stored keys to host memory, w words each, sorted lexicographically
 * by (word0, word1, ...) as unsigned integers (slot padding removed).
 * Waits for all device work.  *n_out receives the number of stored keys.  If
 * host_keys is NULL or cap_states is smaller than that number, nothing is
 * written to host_keys and GX_ENOMEM is returned (with *n_out set).
 */
gx_status gx_table_dump(gx_table* table, uint32_t* host_keys, uint64_t cap_states,
                        uint64_t* n_out);

/* Copy raw bucket storage words [first_word, first_word + n_words) to host
 * memory (for placement checks).  Waits for all device work. */
gx_status gx_table_read_raw(gx_table* table, uint32_t* host_words, uint64_t first_word,
                            uint64_t n_words);

/* Copy raw bucket storage words [first_word, first_word + n_words) into device
 * memory dev_words (caller-owned, on the table's device), e.g. to inspect a
 * table too large for host memory window by window.  Stream-ordered on
 * hip_stream.  Errors: GX_EINVAL (null pointer with n_words > 0, range outside
 * the storage), GX_EDEVICE (the copy could not be queued). */
gx_status gx_table_copy_raw(gx_table* table, uint32_t* dev_words, uint64_t first_word,
                            uint64_t n_words, void* hip_stream);

/*
 * Bucket index that hash function j assigns to a key (host only).  The family
 * is h_j(k) = mulhi64(a_j * m(k) + c_j, n_buckets): m is a 64-bit mix of the
 * key words under the seed, (a_j, c_j) the j-th set of hash constants drawn
 * from the seed, and mulhi64 the high 64 bits of a 128-bit product (a range
 * reduction that needs no power-of-two bucket count).  The paper fixes only
 * that there are H sets of hash constants (8 by default, Sec. 4.1).
 */
gx_status gx_hash_bucket(const uint32_t* key, uint32_t words_per_state, uint64_t hash_seed,
                         uint32_t j, uint64_t n_buckets, uint64_t* bucket);

/* ------------------------------------------------------------ networks */

/* One LTS (Sec. 3): n_states local states 0..n_states-1, an initial state and
 * n_trans transitions (src[i], label[i], dst[i]), host arrays. */
typedef struct {
  uint32_t n_states, initial, n_trans;
  const uint32_t* src;
  const uint32_t* label;
  const uint32_t* dst;
} gx_lts;

/*
 * A network of LTSs with synchronisation rules (Sec. 3, Fig. 1).
 * rules: host, n_rules x n_procs int32, row-major; entry [r][p] is the label
 * process p must take in rule r, or -1 if p does not take part.  A transition
 * of process p whose label is named at position p by some rule fires only
 * through rules (all participants step together, one product transition per
 * choice of matching transitions); every other transition fires alone.
 */
typedef struct {
  uint32_t n_procs;
  const gx_lts* procs;
  uint32_t n_labels;
  uint32_t n_rules;
  const int32_t* rules;
} gx_network;

/*
 * Words per packed state vector (Sec. 3: process states are combined in
 * 32-bit integers; Sec. 5.2: longer vectors take several integers).  Field
 * width of process p is max(1, ceil(log2 n_states)); fields are placed in
 * process order from bit 0, a field that would cross bit 31 starts the next
 * word, and bit 31 of every word stays 0.  Errors: GX_EINVAL for an invalid
 * network or more than 4 words.
 */
gx_status gx_network_words(const gx_network* net, uint32_t* words_per_state);

/* Pack n host vectors of local states (n x n_procs uint32) into n x w words
 * (host only). */
gx_status gx_network_pack(const gx_network* net, const uint32_t* local, uint64_t n,
                          uint32_t* out);

/*
 * Automaton of a negated safety property (Sec. 3: such an automaton can be
 * added to the network, and reaching one of its bad states during the
 * exploration shows that the property is violated).  It observes actions of
 * the network, numbered as follows: action r < n_rules is synchronisation
 * rule r; action n_rules + l is label l fired alone by any process.
 */
typedef struct {
  uint32_t n_states, initial, n_trans;
  const uint32_t* src;     /* host, n_trans                                  */
  const uint32_t* action;  /* host, n_trans: the action observed             */
  const uint32_t* dst;     /* host, n_trans                                  */
  const uint8_t* bad;      /* host, n_states: nonzero = bad state            */
} gx_monitor;

/* A network with a monitor as its last process (library-owned arrays). */
typedef struct {
  gx_network net;              /* pass to gx_network_words and gx_explore    */
  uint32_t monitor_proc;       /* the automaton's process index (n_procs - 1) */
  const uint8_t* monitor_bad;  /* its bad-state flags, for gx_explore_opts    */
  void* owner;                 /* library-internal                            */
} gx_monitored_network;

/*
 * Add a safety monitor to a network (Sec. 3), host only.  The automaton
 * becomes one more process: a rule it observes gains it as a participant,
 * and a label it observes that process p fires alone becomes a rule of p and
 * the automaton (one rule per such process), each observed action with a
 * label of its own; unobserved actions fire as before.  Where the automaton
 * leaves an observed action unspecified in some state it stays in that state
 * (it never blocks the network); observed actions the network never
 * performs are dropped.  Explore the result with opts.monitor_proc =
 * out->monitor_proc and opts.monitor_bad = out->monitor_bad; free it with
 * gx_monitored_network_free.  Errors: GX_EINVAL (invalid network or
 * automaton, an action out of range), GX_ENOMEM.
 */
gx_status gx_network_add_monitor(const gx_network* net, const gx_monitor* mon,
                                 gx_monitored_network* out);

/* Release what gx_network_add_monitor allocated.  NULL is accepted. */
void gx_monitored_network_free(gx_monitored_network* m);

typedef struct {
  uint64_t frontier_capacity; /* largest BFS level (states) the call may buffer;
                                 0 -> limited by device memory only           */
  uint64_t deadlock_capacity; /* largest deadlock count the call may buffer;
                                 0 -> limited by device memory only           */
  void* hip_stream;           /* stream for every launch of the call           */
  uint32_t local_dedup;       /* nonzero: before probing the table, each
                                 wavefront drops duplicates within its staged
                                 chunk of successors (the per-block state cache
                                 of the paper's tool, Sec. 3); results are
                                 unchanged, table probes fewer                 */
  uint32_t monitor_proc;      /* with monitor_bad: the process that is the
                                 automaton of a negated safety property (Sec. 3) */
  uint32_t stop_on_violation; /* nonzero: end the exploration after the first
                                 level that holds a violation (that level is
                                 counted, not expanded)                        */
  uint32_t slice_states;      /* most frontier states one slice of a level
                                 takes (one generation launch, then one probe
                                 launch, whose successor buffer holds the
                                 slice's successors); 0 -> 2^22               */
  const uint8_t* monitor_bad; /* host, n_states of monitor_proc bytes, nonzero
                                 = bad local state; NULL: no safety check      */
} gx_explore_opts;

typedef struct {
  uint64_t n_states;      /* reachable states                                  */
  uint64_t n_transitions; /* product transitions of the reachable states       */
  uint32_t words_per_state;
  uint32_t n_levels;      /* BFS levels; level 0 is the initial state          */
  uint64_t* level_counts; /* n_levels entries (library-owned)                  */
  uint64_t n_deadlocks;   /* reachable states without a product transition     */
  uint32_t* deadlocks;    /* n_deadlocks x w words, sorted (library-owned)     */
  uint64_t local_duplicates; /* successors dropped by the local duplicate
                                filter (gx_explore with local_dedup), else 0  */
  uint64_t n_violations;  /* reachable states (of the levels found) whose
                             monitor process is in a bad state; 0 without a
                             monitor                                           */
  uint32_t* violations;   /* n_violations x w words, sorted (library-owned)    */
  uint32_t violation_level; /* first level holding a violation; 0xFFFFFFFF
                               when none                                      */
  uint32_t reserved;
  uint32_t* states;       /* the reachable states (the table's contents),
                             n_states x w words, sorted (library-owned); only
                             when asked for (keep_states of a batch or a
                             server), else NULL                               */
} gx_explore_result;

/*
 * Breadth-first exploration of the synchronous product (Sec. 3), level by
 * level, with on-the-fly deadlock detection.  Every successor goes through
 * the table's find-or-put; states it reports NEW form the next level.
 *
 *   net    host description; compiled to a device image for the call.
 *   table  caller-created, empty (nothing inserted since its creation or
 *          its last gx_table_clear; else GX_EINVAL before any device work),
 *          with words_per_state equal to gx_network_words(net); it holds the
 *          reachable set afterwards.
 *   opts   nullable.
 *   out    filled on success; free with gx_explore_result_free.
 *
 * Device buffers (frontiers, successor buffer, deadlock list, network image)
 * are owned by the table, allocated on first use and grown on demand; later
 * explorations into the same table reuse them.  A level is expanded in
 * slices sized so that neither the next frontier nor the successor buffer
 * can overflow even if every successor were new; each slice is one
 * successor-generation launch followed by one find-or-put-and-append launch
 * on opts->hip_stream.  The network image (the transition tables of every
 * process and rule, about one word per local state and transition) is read
 * from LDS when it fits 11776 words (46 KiB), else from global memory (up to
 * 2^26 words; such networks skip the small-level path).
 *
 * Safety check (Sec. 3: the negation of a safety property is an automaton
 * added to the network as one more process): with opts->monitor_bad set, a
 * state whose local state of process opts->monitor_proc is marked bad is a
 * violation.  Each level is scanned as soon as it is complete (one extra
 * streaming pass over it); violations and the first level holding one are
 * returned, and with opts->stop_on_violation the exploration ends there
 * (that level is counted, not expanded; the table holds the states of the
 * levels returned).
 *
 * Synchronous: returns when the exploration ends.
 * Errors: GX_EINVAL (invalid network, word count mismatch, non-empty table,
 * network image above 2^26 words, monitor_proc out of range),
 * GX_ETABLEFULL (a state
 * exhausted every hash function; exploration stops, no result), GX_ENOMEM
 * (frontier or deadlock buffer too small, or allocation failure).
 */
gx_status gx_explore(const gx_network* net, gx_table* table, const gx_explore_opts* opts,
                     gx_explore_result* out);

/* Release the arrays of a result filled by gx_explore.  NULL is accepted. */
void gx_explore_result_free(gx_explore_result* result);

/* ------------------------------------------------- exploration, no allocation */

/* Device memory of gx_explore_noalloc: one array of this size per GPU the
 * library runs on, held until the process ends. */
#define GX_NOALLOC_SCRATCH_BYTES (64u << 20)

typedef struct {
  uint64_t n_states, n_transitions;
  uint32_t n_levels, words_per_state;
  uint64_t n_deadlocks;
} gx_explore_summary;

/*
 * For callers that cannot allocate (code near HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): gx_explore with every
 * device buffer it needs beyond the table in the library's static scratch
 * array of GX_NOALLOC_SCRATCH_BYTES on the current device, and the results in
 * the caller's host arrays.  It calls no hipMalloc, hipHostMalloc or hipFree
 * and returns nothing that needs freeing.
 *
 *   net, table, opts  as for gx_explore (the table must be on the current
 *                device; no safety monitor: opts->monitor_bad must be NULL).
 *   level_counts  host, max_levels entries (max_levels >= 1): the level counts.
 *   deadlocks     host, max_deadlocks x w words (nullable when max_deadlocks
 *                 is 0): the deadlock states, sorted.
 *   out           the counts.
 *
 * The scratch array holds a 64 KiB control block and four equal buffers of
 * (GX_NOALLOC_SCRATCH_BYTES - 65792) / 4 bytes rounded down to a multiple of
 * 256 (two frontiers, successors, deadlocks): 4,190,144 states of a 1-word
 * slot, 2,095,072 of 2 words, 1,047,536 of 4 (3-word states take 4-word
 * slots).
 * A level, the successors of one state or the deadlocks beyond that, or more
 * levels or deadlocks than the caller's arrays hold, give GX_ENOMEM (the
 * table keeps what was stored).  Every call on a GPU uses that GPU's one
 * array: calls that overlap on one GPU (two host threads, or two streams)
 * race and must be serialised by the caller.  Synchronous.
 * Errors: as gx_explore, plus GX_EINVAL for a monitor, null arrays, a
 * table on another device or a network image beyond the 46 KiB the control
 * block holds.
 */
gx_status gx_explore_noalloc(const gx_network* net, gx_table* table, const gx_explore_opts* opts,
                             uint64_t* level_counts, uint32_t max_levels, uint32_t* deadlocks,
                             uint64_t max_deadlocks, gx_explore_summary* out);

/* Static string naming a status code. */
const char* gx_status_str(gx_status status);

/* ------------------------------------------------------------ batches */

/*
 * Batched exploration: many networks (instances) explored together, each
 * with its own table partition carved from one allocation per kernel class.
 * Every instance follows exactly the single-exploration semantics of
 * gx_explore (Sec. 3).  Instances that share a kernel configuration (slot
 * words, bucket words, subgroup, keys per subgroup) form a class.  Two
 * schedules:
 *   stepped (the default): every unfinished instance advances one BFS level
 *     per step; a step is one launch per class over the current levels of
 *     all its unfinished instances, then one read-back of their next-level
 *     sizes.  gx_batch_run drives the steps from the calling thread and
 *     returns when every instance has finished.
 *   persistent (use_graph or persistent nonzero): one persistent launch per
 *     class, classes concurrently on their own streams; instances advance
 *     independently, workgroups pulling (instance, level, tile) work from a
 *     device-side queue; gx_batch_run only enqueues, and a whole run can be
 *     captured in a hipGraph.
 */
typedef struct gx_batch gx_batch;

typedef struct {
  const uint64_t* capacity;   /* host, n entries, required: table capacity
                                 (states) of each instance; also the size of
                                 its two frontier buffers                     */
  uint64_t hash_seed;         /* 0 -> the default seed                         */
  uint32_t max_hashes;        /* H; 0 -> 8                                     */
  uint32_t bucket_words;      /* 0 -> autotuned per instance: the pick of
                                 gx_autotune_capacity for its words, load 0.5
                                 and the sum of the capacities of the
                                 instances of its slot width (their tables
                                 share the caches while they run together);
                                 else 8|16|32|64                              */
  uint32_t subgroup;          /* 0 -> autotuned per instance, else 4|8|16
                                 (4 with buckets of at most 32 words; an
                                 explicit 4 caps an autotuned bucket at 32)   */
  uint32_t keys_per_subgroup; /* 0 -> 1, else 1|2                             */
  uint32_t use_graph;         /* nonzero: the persistent schedule, and
                                 gx_batch_create captures a whole run (clears,
                                 resets and every launch) in a hipGraph that
                                 gx_batch_run replays                         */
  uint32_t max_levels;        /* BFS levels per instance; 0 -> 4096.  An
                                 instance deeper than this gets GX_ENOMEM.  In
                                 the persistent schedule the device work queue
                                 holds instances x max_levels entries of 32
                                 bytes, so every level of every instance fits;
                                 instances x max_levels must then stay below
                                 2^31 (else GX_EINVAL)                        */
  uint64_t deadlock_capacity; /* deadlock records per class; 0 -> min(sum of
                                 capacities, 2^26)                             */
  void* hip_stream;           /* stream used by gx_explore_batch               */
  uint32_t keep_states;       /* nonzero: gx_batch_results also returns every
                                 instance's reachable states (its table
                                 partition's contents) in outs[i].states      */
  uint32_t persistent;        /* nonzero: the persistent schedule without a
                                 graph; 0 (and use_graph 0): stepped          */
} gx_batch_opts;

/* Compile every network (argument errors before device work, GX_EINVAL also
 * for a network image beyond the 46 KiB of LDS the batch kernels keep it
 * in), choose each instance's kernel configuration, allocate and upload.
 * Synchronous. */
gx_status gx_batch_create(const gx_network* nets, uint32_t n, const gx_batch_opts* opts,
                          gx_batch** out);

/* Clear every table and explore every instance from its initial state, on
 * hip_stream after the work already queued there.  Stepped schedule: returns
 * when the run has finished (the calling thread drives its steps).
 * Persistent schedule: enqueues the run and returns.  May be called again to
 * repeat the whole batch. */
gx_status gx_batch_run(gx_batch* batch, void* hip_stream);

/* Wait for the last run and fill outs[i] / inst_status[i] for every instance
 * (GX_OK, GX_ETABLEFULL, GX_ENOMEM when a frontier, level or deadlock buffer
 * was too small, GX_EDEVICE when the run was aborted).  outs of instances
 * with GX_OK are freed with gx_explore_result_free.  Returns GX_EINVAL before
 * any run. */
gx_status gx_batch_results(gx_batch* batch, gx_explore_result* outs, gx_status* inst_status);

/* Kernel configuration chosen for instance i (host only). */
gx_status gx_batch_instance_config(const gx_batch* batch, uint32_t i, uint32_t* bucket_words,
                                   uint32_t* subgroup, uint32_t* keys_per_subgroup);

gx_status gx_batch_destroy(gx_batch* batch);

/* create + run + results + destroy. */
gx_status gx_explore_batch(const gx_network* nets, uint32_t n, const gx_batch_opts* opts,
                           gx_explore_result* outs, gx_status* inst_status);

/*
 * Autotuner: the kernel configuration (bucket words, subgroup; one key in
 * flight per subgroup, as the exploration kernels keep) for tables of
 * words_per_state-word states filled to load_factor (0 < load_factor <=
 * 0.95), per size class of the table's capacity (up to 2^16, 2^20, 2^24
 * states, and larger: the class decides whether its buckets live in an
 * XCD's L2, the last-level cache or HBM).  The first call for a (slot words,
 * load, size class) times every candidate (B in 8..64, subgroup 4 (B <= 32),
 * 8 or 16) on a stream shaped like an exploration's successor lookups (every
 * distinct key about 8 times, shuffled; at least 2^25 keys per measurement,
 * the median of three) into a table at the top of the class, and picks the
 * fastest, except that the default (B = 16, subgroup 4) is kept when it is
 * within 3% of the fastest; later calls return the cached choice.
 * Synchronous.
 */
typedef struct {
  uint32_t bucket_words, subgroup, keys_per_subgroup;
  uint32_t candidates;         /* configurations timed                        */
  double ns_per_key;           /* the pick's time per key                     */
  double ns_per_key_default;   /* the default's (B = 16, subgroup 4)          */
  double ns_per_key_runner_up; /* the fastest candidate other than the pick:
                                  the decision margin is runner_up / pick - 1
                                  (negative when a near-tie kept the default) */
  uint64_t table_slots;        /* size of the timed table                     */
  uint32_t size_class;         /* 0..3                                        */
  uint32_t pad;
} gx_tune_info;

gx_status gx_autotune_capacity(uint32_t words_per_state, double load_factor, uint64_t capacity,
                               gx_tune_info* info);

/* The pick of gx_autotune_capacity for a table of 2^23 / load_factor states
 * (the size class of 2^23 states at that load). */
gx_status gx_autotune(uint32_t words_per_state, double load_factor, uint32_t* bucket_words,
                      uint32_t* subgroup, uint32_t* keys_per_subgroup);

/* ------------------------------------------------------------ serving */

/*
 * Exploration server.  Requests (a network and a declared bound on its number
 * of reachable states) are admitted when their HBM reservation fits the
 * budget: a table with ceil(bound / load_factor) slots rounded up to a power
 * of two, two frontier buffers and a deadlock buffer of as many states, one
 * power-of-two block of a device arena of budget_bytes that the server
 * allocates once at creation (a buddy allocator: admission allocates
 * nothing; the largest reservation that can ever fit is the largest power
 * of two within the budget).  A host thread runs steps: one launch per slot width
 * expands the current BFS level of every admitted request, so requests that
 * arrive while others run join at the next step (continuous batching).  A
 * request whose table fills up is retried with four times its bound (at
 * least twice the states found before it filled up; up to 12 attempts, and
 * only while the reservation fits the budget).  Results equal those of gx_explore on the same network.
 */
typedef struct gx_server gx_server;

typedef struct {
  uint64_t budget_bytes;      /* HBM of the server's arena (tables, frontiers),
                                 allocated at creation                         */
  uint32_t max_active;        /* requests admitted at once; 0 -> 256           */
  uint32_t max_hashes;        /* H; 0 -> 8                                     */
  double load_factor;         /* table load at the declared bound; 0 -> 0.5   */
  uint64_t hash_seed;         /* 0 -> the default seed                         */
  uint32_t bucket_words;      /* 0 -> autotuned per slot width, else 8..64     */
  uint32_t subgroup;          /* 0 -> autotuned, else 4|8|16 (4 with buckets
                                 of at most 32 words)                         */
  uint32_t keys_per_subgroup; /* 0 -> 1, else 1|2                             */
  uint32_t keep_states;       /* nonzero: a completed request's result also
                                 holds its reachable states (its table's
                                 contents, read before the table is released)
                                 in result.states                              */
} gx_server_opts;

typedef struct {
  uint64_t submitted, completed, failed, retried;
  uint64_t steps;          /* multi-request launches run                        */
  uint64_t active_peak;    /* largest number of requests admitted at once       */
  uint64_t reserved_peak;  /* largest reservation held (bytes)                  */
  uint64_t states;         /* reachable states of completed requests            */
  uint64_t reserved_now, pooled_bytes /* arena bytes not reserved */, waiting;
} gx_server_stats;

/* Start a server on the current device (spawns its step thread). */
gx_status gx_server_create(const gx_server_opts* opts, gx_server** out);

/* Queue a request; the network is compiled and copied before return.
 * Errors: GX_EINVAL (invalid network, a network image beyond the 46 KiB of
 * LDS the step kernel keeps it in, bound 0). */
gx_status gx_server_submit(gx_server* server, const gx_network* net, uint64_t declared_states,
                           uint64_t* request_id);

/* Result of a request.  wait = 0: GX_EBUSY while it runs.  On GX_OK the
 * request's status (GX_OK, GX_ETABLEFULL after the last retry, GX_ENOMEM when
 * it can never fit the budget, GX_EDEVICE), its result (owned by the caller,
 * gx_explore_result_free) and its latency from submission to completion are
 * returned, and the request is forgotten. */
gx_status gx_server_poll(gx_server* server, uint64_t request_id, int wait,
                         gx_explore_result* out, gx_status* request_status,
                         uint64_t* latency_ns);

gx_status gx_server_get_stats(gx_server* server, gx_server_stats* out);

/* Stop the step thread and free everything; no other call on the server may
 * overlap it. */
gx_status gx_server_destroy(gx_server* server);

/* ------------------------------------------------------------ measurement */

/*
 * Random-access bandwidth probe: n_reads reads of `granule` bytes (4..256,
 * power of two) at pseudo-random granule-aligned offsets of a device buffer of
 * buf_bytes bytes (buf_bytes >= granule), one subgroup of granule/4 lanes (at
 * most 64) per read; the sum of the values read is written to *sink (device,
 * 8 bytes) so the reads cannot be removed.  Stream-ordered.  Gives the
 * achievable random-access bandwidth that bounds the table probes.
 */
gx_status gx_gather_probe(const uint32_t* buf, uint64_t buf_bytes, uint32_t granule,
                          uint64_t n_reads, uint64_t seed, uint64_t* sink, void* hip_stream);

/*
 * Claim probe: n_ops operations at pseudo-random 64-byte-aligned offsets of
 * a device buffer of buf_bytes bytes (>= 64, 64-byte aligned).  mode 1: one
 * device-scope 64-bit compare-and-swap each (the claim of a find-or-put,
 * Sec. 4.1); mode 2: an 8-byte read each and, for every other operation, a
 * compare-and-swap in the granule just read (a find-or-put of keys half of
 * which are new).  The buffer's contents are changed; a value derived from
 * them is added to *sink (device, 8 bytes).  Stream-ordered.  Gives the
 * ceiling that claims put on find-or-put.  Errors: GX_EINVAL (null, too
 * small or misaligned buffer, other modes), GX_EDEVICE (launch).
 */
gx_status gx_claim_probe(uint64_t* buf, uint64_t buf_bytes, uint32_t mode, uint64_t n_ops,
                         uint64_t seed, uint64_t* sink, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* GX_H */
