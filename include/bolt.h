/*
 * bolt.h - C ABI of an oblivious key-value map on one AMD Instinct MI355X
 * (gfx950), after BOLT (arxiv 2509.01742).
 *
 * The map splits K + M logical bins between the GPU's HBM (K bins, never
 * observable) and an observable store of M fixed-size pages (pinned host
 * memory reached over the host link, or a designated device buffer).  Every
 * key sits in one of two random bins, the less loaded one (Sec. 4.1, Alg. 1).
 * A lookup reads both bins whole and then moves the key to two fresh random
 * bins, so the observable store sees two uniformly random bins per command
 * whatever the keys, values and commands are (Claim 4.1).
 *
 * Conventions for every call below
 *   - Pointers named d_* are device pointers (for example a torch tensor's
 *     data_ptr()) owned by the caller; they must stay valid until the stream
 *     reaches the call.  Host pointers are named host_* and are used before
 *     the call returns.
 *   - hip_stream is a hipStream_t (NULL = the legacy default stream).  Calls
 *     are ordered on the stream and return before the device work ends;
 *     results are valid after the stream has been synchronised.  Calls on one
 *     map must not overlap from several host threads.
 *   - A negative return is an error.  Argument errors are reported at once and
 *     change nothing.  Errors found on the device (capacity overflow, duplicate
 *     build keys, live keys beyond capacity) are sticky: bolt_status() reports
 *     them after synchronising, and from then on the map is poisoned and every
 *     call except bolt_destroy returns BOLT_ESTATE.
 *   - Keys are any 64-bit values.  Values are value_bytes bytes each, rows of
 *     a row-major [q][value_bytes] array.
 *   - The observable pages a batch rewrites (Sec. 5.1 step 5) are rebuilt in
 *     HBM and written to the store during the map's next batch, while that
 *     batch reads its own pages (the host link carries both directions at
 *     once); bolt_flush writes them at once.  Answers never depend on it, and
 *     every call below that reads the store, and bolt_status, flush first.
 */
#ifndef BOLT_H
#define BOLT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bolt_map bolt_map; /* opaque, owned by the library */

/* Return codes. */
enum {
  BOLT_OK = 0,
  BOLT_EINVAL = -1,    /* bad argument, or a call in the wrong state */
  BOLT_ENOMEM = -2,    /* device or pinned host allocation failed */
  BOLT_EDUPKEY = -3,   /* bolt_build got the same key twice (keys are unique, Sec. 2.1) */
  BOLT_EOVERFLOW = -4, /* a bin, stash or position-map row would exceed its capacity */
  BOLT_EFULL = -5,     /* live keys would exceed the capacity (or the trace log is full) */
  BOLT_EHIP = -6,      /* a HIP runtime call failed */
  BOLT_ESTATE = -7,    /* the map is poisoned by an earlier device-side error */
  BOLT_ETIMEOUT = -8,  /* a server wait ended before the work did */
  BOLT_ETAMPER = -9    /* BOLT_F_SEAL: an observable page or its tag was changed or replayed */
};

/* Operation codes of a command <opcode | key | payload> (Sec. 5.1 step 2).
 * A delete is the paper's PUT with a tombstone payload, given its own code
 * so that every value stays usable. */
enum { BOLT_OP_GET = 0, BOLT_OP_PUT = 1, BOLT_OP_DEL = 2 };

/* Per-command status byte of the fixed-length response (Sec. 5.1 step 6). */
enum {
  BOLT_ST_ABSENT = 0,   /* GET or DEL of a key that was not present */
  BOLT_ST_FOUND = 1,    /* GET of a present key */
  BOLT_ST_UPDATED = 1,  /* PUT of a present key */
  BOLT_ST_INSERTED = 2, /* PUT of an absent key */
  BOLT_ST_DELETED = 3   /* DEL of a present key */
};

/* Where the M observable pages live. */
enum { BOLT_OBS_HOST_PINNED = 0, BOLT_OBS_DEVICE = 1 };

/* bolt_params.flags */
#define BOLT_F_TRACE 1u     /* record every observable access (tests; costs a little time) */
#define BOLT_F_FIXED_KEY 2u /* use params.key as the PRF key instead of fresh OS randomness */
#define BOLT_F_TIMING 4u    /* time every kernel class with HIP events on its stream (benchmarks) */
#define BOLT_F_WATCH 16u    /* after every batch, record the largest bin load and the items held by the HBM bins,
                               with their high-water marks (dynamics validation; one small kernel per batch) */
#define BOLT_F_SEAL 32u     /* seal every observable page: ChaCha20-Poly1305 (RFC 8439) under the nonce
                               LE32(page) || LE64(its write count, kept in HBM); a page read whose tag does
                               not check poisons the map with BOLT_ETAMPER.  Pages up to 8 KiB. */
#define BOLT_F_GRAPHS 8u    /* run one-map batches by replaying a HIP graph captured once per power-of-two batch
                               size (fewer host launch calls; results identical).  Not with TIMING. */
#define BOLT_F_SEAL_CMDS 128u /* commands and responses cross the host sealed: bolt_access_sealed and
                               bolt_server_submit_sealed take ChaCha20-Poly1305 records under params.session_key */
#define BOLT_F_DECOMPOSED 256u /* the decomposed HBM store of Sec. 5.2: the HBM bins' items are value-pool
                               entries listed under their bin (the reverse index), allocated from a free-address
                               ring; no dummy-padded HBM pages.  Results, pages and trace as without it. */
#define BOLT_F_SEAL_KEY_REUSE 64u /* tests only: allow BOLT_F_SEAL together with BOLT_F_FIXED_KEY.  The page key
                               derives from the PRF key and every build starts the write counts at 1, so two maps
                               sealed under one fixed key (or a map re-created with its key) encrypt with the same
                               key streams and Poly1305 keys: their pages leak XORs of plain texts and accept
                               forged tags.  Without this flag bolt_create refuses SEAL with FIXED_KEY. */

#define BOLT_MAX_BATCH 8192u /* most commands in one access call */

typedef struct {
  uint64_t capacity;       /* N_max: most live keys the map will hold */
  uint32_t value_bytes;    /* vs: bytes per value, a multiple of 8; a page (8 + Z (8 + vs) bytes) must fit 32 KiB */
  uint32_t c;              /* mean bin load N/(K+M) (Claim 4.2); the paper's default is 8 */
  uint32_t alpha_permille; /* alpha = K/(K+M) in 1/1000 (Claim 4.4); default 200, below 1000 */
  uint32_t bin_slots;      /* Z, items per bin; 0 = l_max = c + ceil(log2 ceil(log2 N_max)) + 1 (Claim 4.2), plus
                              one when B <= 64 * BOLT_MAX_BATCH (a batch can fill 1/64 of a placement round) */
  uint32_t pm_choices;     /* d, position-map rows a key may use (Sec. 5.2); 1..4, default 4 */
  uint32_t pm_keys_per_row;/* N_max / rows of the position map (Sec. 5.2); default 16 */
  uint32_t pm_row_slots;   /* slots per position-map row, 1..32; default 32 */
  uint32_t observable;     /* BOLT_OBS_* */
  uint32_t flags;          /* BOLT_F_* */
  uint64_t trace_words;    /* capacity of the trace log in 32-bit words (BOLT_F_TRACE) */
  uint8_t key[32];         /* PRF key when BOLT_F_FIXED_KEY is set */
  uint8_t session_key[32]; /* BOLT_F_SEAL_CMDS: the key the user and the map share for command and response
                              records.  It stands in for a key provisioned into the device by attestation,
                              which the paper assumes and does not build; it is copied to device memory at
                              bolt_create. */
} bolt_params;

/* Sizes the library derives from the parameters (all integers). */
typedef struct {
  uint64_t B;           /* bins K + M = ceil(N_max / c) */
  uint64_t K;           /* HBM bins = floor(alpha_permille * B / 1000) */
  uint64_t M;           /* observable pages = B - K */
  uint64_t Z;           /* items per bin (page capacity) */
  uint64_t page_bytes;  /* bytes per page: u64 valid mask, Z keys, Z values, zero pad to 128 */
  uint64_t pm_rows;     /* position-map rows = ceil(N_max / pm_keys_per_row) */
  uint64_t stash_bound; /* ceil((1 + alpha) M / 2 + l_max sqrt(M ln N_max)) (Claim 4.4, constant 1) */
  uint64_t stash_pool;  /* value-pool entries: stash_bound + BOLT_MAX_BATCH, plus hbm_bound when decomposed */
  uint64_t lmax;        /* l_max = c + ceil(log2 ceil(log2 N_max)) + 1, the bound of Claim 4.2 (constant 1) */
  uint64_t hbm_bound;   /* ceil(K c + l_max sqrt(K ln N_max)): items the HBM bins may hold (Claim 4.3) */
} bolt_sizes;

/* Fills p with the paper's defaults (c = 8, alpha = 0.2, d = 4, 16 keys per
 * row, 32 slots) for the given capacity and value size.  No allocation. */
void bolt_params_default(bolt_params* p, uint64_t capacity, uint32_t value_bytes);

/* Derives the sizes of p.  Returns BOLT_EINVAL for parameters out of range. */
int bolt_sizes_of(const bolt_params* p, bolt_sizes* out);

/* Device (HBM) bytes and observable-store bytes one map with parameters p
 * allocates: the analogue of the HBM-usage bound of Claim 5.2 for this
 * layout.  Used to admit maps against an HBM budget.  Either pointer may be
 * NULL. */
int bolt_footprint(const bolt_params* p, uint64_t* hbm_bytes, uint64_t* obs_bytes);

/* Creates an empty, unbuilt map on the current HIP device: allocates all
 * state (Sec. 5.1 step 1) and derives the PRF key.  *out receives the map.
 * Returns BOLT_EINVAL, BOLT_ENOMEM or BOLT_EHIP on failure (nothing leaks). */
int bolt_create(const bolt_params* p, void* hip_stream, bolt_map** out);

/* Oblivious build of the map from n distinct keys d_keys[n] and values
 * d_vals[n][value_bytes] (n <= capacity, n may be 0).  This is the paper's
 * data initialization (Sec. 5.2, "fast data initialization") done on the
 * device without a trusted data owner: a keyed PRF gives each key two bins,
 * P2C places it, a bitonic sorting network and a shift network lay the items
 * into dummy-padded bins, and the pages are written in order 0..M-1, so the
 * observable store sees the same writes for every dataset of size n.
 * Once per map.  Duplicate keys end in BOLT_EDUPKEY (sticky). */
int bolt_build(bolt_map* m, const uint64_t* d_keys, const void* d_vals, uint64_t n, void* hip_stream);

/* Runs q <= BOLT_MAX_BATCH commands in one batch (Alg. 1 per command, Sec. 5.1
 * steps 2-6).  d_ops[q] holds BOLT_OP_* codes, d_keys[q] the keys,
 * d_vals_in[q][vs] the PUT payloads (read for PUT commands only, but always
 * required).  Outputs: d_vals_out[q][vs] gets the value of each GET of a
 * present key and zeros otherwise (fixed-length responses); d_status[q] gets
 * a BOLT_ST_* byte.  The answers equal running the commands one at a time in
 * index order.  Every command reads two whole bins; each page read is written
 * back once at the end of the batch.  Op codes are checked on the device: a
 * batch holding a code above BOLT_OP_DEL is rejected whole, leaves the map
 * unchanged and reports status 0xFF for every command.  d_keys, d_vals_in and
 * d_vals_out must be 8-byte aligned. */
int bolt_access_batch(bolt_map* m, const uint8_t* d_ops, const uint64_t* d_keys, const void* d_vals_in,
                      void* d_vals_out, uint8_t* d_status, uint32_t q, void* hip_stream);

/* q GETs: d_vals_out[q][vs] gets each value (zeros when absent), d_found[q]
 * gets 1 when the key was present and 0 otherwise. */
int bolt_get_batch(bolt_map* m, const uint64_t* d_keys, uint32_t q, void* d_vals_out, uint8_t* d_found,
                   void* hip_stream);

/* q PUTs of d_vals[q][vs]; d_status[q] gets BOLT_ST_UPDATED or BOLT_ST_INSERTED. */
int bolt_put_batch(bolt_map* m, const uint64_t* d_keys, const void* d_vals, uint32_t q, uint8_t* d_status,
                   void* hip_stream);

/* Builds `count` distinct, not yet built maps (all on the current device)
 * from their own key/value arrays: map i from d_keys[i], d_vals[i] and n[i],
 * with the layout and errors of bolt_build.  Every phase of the build runs as
 * one launch for all maps (map = second grid dimension), so many small maps
 * cost about as many launches as the largest one alone.  Each map ends
 * exactly as bolt_build would leave it.  Arguments are checked for every
 * map before anything runs; a map may appear once per call. */
int bolt_build_many(bolt_map* const* maps, const uint64_t* const* d_keys, const void* const* d_vals,
                    const uint64_t* n, uint32_t count, void* hip_stream);

/* One batch of commands for one map (the arguments of bolt_access_batch). */
typedef struct {
  const uint8_t* d_ops;
  const uint64_t* d_keys;
  const void* d_vals_in;
  void* d_vals_out;
  uint8_t* d_status;
  uint32_t q;
} bolt_batch;

/* Runs one batch on each of `count` distinct maps (all on the current
 * device), every phase of the access path as one launch for all of them.
 * Each map gets exactly the result bolt_access_batch would give it; maps of
 * any size and batches of any size up to BOLT_MAX_BATCH mix freely.  This is
 * the multi-map batching of the build's systems layer: it removes the
 * per-map launch cost that dominates small maps and small batches.  A map
 * may appear once per call.  Batches with q = 0 are skipped. */
int bolt_access_many(bolt_map* const* maps, const bolt_batch* batches, uint32_t count, void* hip_stream);

/* BOLT_F_SEAL maps: the tags (M x 16 bytes, observable, beside the pages)
 * and the write count of every page (M x u64, in HBM). */
int bolt_tags_snapshot(bolt_map* m, void* host_buf, uint64_t cap);
int bolt_versions_snapshot(bolt_map* m, uint64_t* host_buf, uint64_t cap);

/* BOLT_F_SEAL maps: what an adversary holding the observable store can do,
 * for tests.  Reads (write = 0) or overwrites (write = 1) page `page` and its
 * tag: host_buf holds page_bytes + 16 bytes.  Synchronises first. */
int bolt_observable_raw(bolt_map* m, uint64_t page, void* host_buf, int write);

/* Writes the observable pages rebuilt by the map's last batch to the store
 * (a no-op when there are none), ordered on hip_stream, which must be the
 * stream of the map's last call or ordered after it.  Needed only where the
 * store itself is read from outside the library. */
int bolt_flush(bolt_map* m, void* hip_stream);

/* Frees every resource of the map after waiting for its work.  NULL is a no-op. */
int bolt_destroy(bolt_map* m);

/* Synchronises the map's last stream and returns BOLT_OK or the sticky
 * device-side error (BOLT_ETAMPER before BOLT_EOVERFLOW before BOLT_EDUPKEY
 * before BOLT_EFULL).  Overflow is the event Sec. 4.3 bounds (a bin above
 * its capacity, the stash above the Claim 4.4 bound, a position-map row
 * full): the paper accepts it as rare data loss; here it is never silent
 * and poisons the map. */
int bolt_status(bolt_map* m);

/* Derived sizes of an existing map. */
int bolt_map_sizes(const bolt_map* m, bolt_sizes* out);

/* Counters of an existing map (synchronises first). */
typedef struct {
  uint64_t live;            /* keys present */
  uint64_t steps;           /* commands run so far (the tape counter) */
  uint64_t batches;         /* access batches run */
  uint64_t stash_live;      /* items in the eviction stash */
  uint64_t stash_highwater; /* largest stash_live seen at the end of a batch */
  uint32_t max_load;        /* largest bin load now */
  uint32_t max_row;         /* fullest position-map row now */
  uint32_t load_highwater;  /* BOLT_F_WATCH: largest bin load seen at a batch end (else 0) */
  uint64_t hbm_load;        /* BOLT_F_WATCH: items in the K HBM bins at the last batch end */
  uint64_t hbm_load_highwater; /* BOLT_F_WATCH: largest hbm_load seen */
} bolt_stats;
int bolt_get_stats(bolt_map* m, bolt_stats* out);

/* ---------------------------------------------------------------------
 * Trace and state readout (tests and diagnostics).  All of these
 * synchronise the map's stream first and copy into host memory.
 * --------------------------------------------------------------------- */

/* One observable access.  batch 0 is the build; access batches count from
 * 1 (a rejected batch takes its number and records nothing).  kind 0 = read of a whole page, 1 = write of a whole page.  Within a
 * batch the reads come in command order (two roles per command, HBM bins
 * omitted), then the writes in ascending page order, as one canonical
 * sequence of what the accessor did (the writes of one batch run
 * concurrently on the device). */
typedef struct {
  uint32_t batch;
  uint32_t kind;
  uint64_t page;
} bolt_trace_rec;

/* Copies up to cap records of the trace recorded since create (or the last
 * clear) into host_recs; *n receives the total count.  The trace is what an
 * adversary watching the observable store sees (Def. 3.1; the simulator of
 * Claim 4.1): one record per page read or written, in the canonical order
 * of each batch (reads by command and role, then the writes by ascending
 * page; the build writes pages 0..M-1).  Returns BOLT_EINVAL if the map was
 * created without BOLT_F_TRACE, BOLT_EFULL if the log filled up and records
 * were lost. */
int bolt_trace_read(bolt_map* m, bolt_trace_rec* host_recs, uint64_t cap, uint64_t* n);
int bolt_trace_clear(bolt_map* m);

/* Raw state, for tests: the M observable pages (the untrusted host memory
 * of Sec. 3, after any pending page writes reach it), the K HBM bins (zeros
 * for a decomposed store, which has no HBM pages), the B bin loads (u32;
 * load(b) counts the bin's items and the stash items bound for it, the
 * quantity P2C compares, Sec. 4.1).  cap is the size of the host buffer in
 * bytes; it must hold the whole array. */
int bolt_observable_snapshot(bolt_map* m, void* host_buf, uint64_t cap);
int bolt_hbm_snapshot(bolt_map* m, void* host_buf, uint64_t cap);
int bolt_loads_snapshot(bolt_map* m, uint32_t* host_buf, uint64_t cap);

/* Logical stash: up to cap live entries as (key, destination bin, value);
 * host_vals holds cap * value_bytes bytes.  *n receives the live count. */
int bolt_stash_snapshot(bolt_map* m, uint64_t* host_keys, uint32_t* host_bins, void* host_vals, uint64_t cap,
                        uint64_t* n);

/* Logical position map: up to cap entries as (row, key, p1, p2); *n receives
 * the entry count. */
int bolt_pm_snapshot(bolt_map* m, uint64_t* host_rows, uint64_t* host_keys, uint32_t* host_p1,
                     uint32_t* host_p2, uint64_t cap, uint64_t* n);

/* Per-kernel-class device time of a map created with BOLT_F_TIMING: HIP
 * events recorded on the launch stream around every launch, summed since
 * create or the last reset.  Fills up to cap entries of host_out (name,
 * launches, total milliseconds); *n receives the number of classes.
 * Synchronises the map's stream.  BOLT_EINVAL without BOLT_F_TIMING. */
typedef struct {
  char name[32];
  uint64_t launches;
  double total_ms;
} bolt_kernel_time;
int bolt_kernel_times(bolt_map* m, bolt_kernel_time* host_out, uint32_t cap, uint32_t* n);
int bolt_kernel_times_reset(bolt_map* m);

/* ---------------------------------------------------------------------
 * Serving: many maps resident on the device behind one request loop.
 *
 * The library runs the loop on a thread of its own.  The caller's
 * requests are host buffers (the paper's command and response buffers,
 * Sec. 5.1); the loop copies commands to the device, runs them and copies
 * the responses back into the caller's buffers.
 *   - Admission: a map opened on the server is created and built on the
 *     device when its footprint (bolt_footprint's device bytes plus its
 *     command staging) fits the HBM budget next to the maps already there.
 *     Maps are admitted in the order they were opened; requests to a map
 *     that waits for admission wait with it.  Closing a map returns its
 *     share once its queued requests are done.
 *   - Continuous batching: whenever a map is idle and has queued requests,
 *     the loop takes its queue head, as many whole requests as fit
 *     max_batch commands, in submission order.  Every map taken in one turn
 *     of the loop runs as one bolt_access_many on a free stream; requests
 *     that arrive while groups run go into the next turn, on another stream,
 *     so the work of different maps overlaps on the device.
 *   - Results: the commands of one map run in submission order with the
 *     semantics of bolt_access_batch, so a request's responses are the same
 *     whether it runs alone or among others (requests of other maps never
 *     change them).
 *   - Latency: completion time minus the arrival time given at submission
 *     (bolt_now_ns clock), so time spent waiting for admission, a stream or
 *     the map counts.
 * --------------------------------------------------------------------- */

typedef struct bolt_server bolt_server; /* opaque, owned by the library */

typedef struct {
  uint64_t hbm_budget; /* device bytes the server's maps may hold together (0 = no limit) */
  uint32_t streams;    /* HIP streams for groups in flight at once, 1..16 (0 = 4) */
  uint32_t max_batch;  /* most commands of one map in one launch, 1..BOLT_MAX_BATCH (0 = BOLT_MAX_BATCH);
                          also the largest request */
  uint32_t flags;      /* must be 0 */
} bolt_server_params;

typedef struct {
  uint64_t submitted, completed, failed; /* requests since the last reset */
  uint64_t commands;                     /* commands of the completed requests */
  uint64_t launches;                     /* groups launched */
  uint64_t queued, queue_peak;           /* requests waiting for launch: now, most at once */
  uint64_t maps_admitted;                /* admissions since the last reset */
  uint64_t maps_resident, maps_waiting;  /* now */
  uint64_t hbm_used, hbm_peak;           /* budgeted device bytes: now, most at once */
  double lat_p50_ms, lat_p99_ms, lat_max_ms, lat_mean_ms; /* arrival to completion */
  double span_s;                         /* first arrival to last completion */
  double mean_group_maps, mean_group_commands;
} bolt_server_stats;

/* Map states reported by bolt_server_map_state. */
enum { BOLT_SRV_WAITING = 0, BOLT_SRV_BUILDING = 1, BOLT_SRV_RESIDENT = 2, BOLT_SRV_CLOSED = 3, BOLT_SRV_FAILED = 4 };

/* CLOCK_MONOTONIC in nanoseconds: the clock of arrival times. */
uint64_t bolt_now_ns(void);

/* Device bytes a map with these parameters holds on a server whose batches
 * are at most max_batch commands (0 = BOLT_MAX_BATCH): the amount admission
 * counts against the budget. */
int bolt_server_footprint(const bolt_params* params, uint32_t max_batch, uint64_t* bytes);

/* Starts a server on the current device.  params may be NULL (defaults). */
int bolt_server_create(const bolt_server_params* params, bolt_server** out);

/* Registers a map with its build input (copied before the call returns;
 * host_keys[n], host_vals[n * value_bytes]).  Tracing and timing flags are
 * refused.  BOLT_EFULL if its footprint alone exceeds the budget.  The map
 * is built when admitted; a build error fails its queued requests. */
int bolt_server_open_map(bolt_server* srv, const bolt_params* params, const uint64_t* host_keys,
                         const void* host_vals, uint64_t n, uint32_t* map_id);

/* Closes a map: requests already queued still run; later submits fail. */
int bolt_server_close_map(bolt_server* srv, uint32_t map_id);

/* *state = BOLT_SRV_*; *err (may be NULL) = the error that failed the map. */
int bolt_server_map_state(bolt_server* srv, uint32_t map_id, int* state, int* err);

/* The device map behind map_id while it is resident (NULL otherwise), for
 * inspection between requests; no call on it may overlap the server's work. */
bolt_map* bolt_server_map(bolt_server* srv, uint32_t map_id);

/* Queues a request of q commands (1 <= q <= max_batch) for a map.  The five
 * host buffers are the request's commands and responses, laid out as in
 * bolt_access_batch; they must stay valid until the request completes.
 * Op codes above BOLT_OP_DEL are refused here (BOLT_EINVAL).  arrival_ns = 0
 * stamps the request now.  *ticket names the request. */
int bolt_server_submit(bolt_server* srv, uint32_t map_id, const uint8_t* host_ops, const uint64_t* host_keys,
                       const void* host_vals_in, void* host_vals_out, uint8_t* host_status, uint32_t q,
                       uint64_t arrival_ns, uint64_t* ticket);

/* A sealed request for a map opened with BOLT_F_SEAL_CMDS (Sec. 3 and
 * Sec. 5.1: the host relays only sealed commands and results): q command
 * records in, q response records out (host buffers, valid until the
 * request completes; layout under bolt_access_sealed).  The map's k-th
 * sealed request is request number k of its session.  Such maps take no
 * plain requests (bolt_server_submit returns BOLT_EINVAL for them).  The
 * host cannot read the op codes: a record with one above BOLT_OP_DEL
 * rejects the coalesced batch it runs in, and a record that fails its tag
 * poisons the map (its requests then fail with BOLT_ETAMPER). */
int bolt_server_submit_sealed(bolt_server* srv, uint32_t map_id, const void* host_req_records, uint32_t q,
                              void* host_resp_records, uint64_t arrival_ns, uint64_t* ticket);

/* *result = 1 while the request is pending, else its return code. */
int bolt_server_poll(bolt_server* srv, uint64_t ticket, int* result);

/* Waits for one request: its return code, or BOLT_ETIMEOUT. */
int bolt_server_wait(bolt_server* srv, uint64_t ticket, uint32_t timeout_ms);

/* Waits until every submitted request has finished, or BOLT_ETIMEOUT. */
int bolt_server_drain(bolt_server* srv, uint32_t timeout_ms);

int bolt_server_get_stats(bolt_server* srv, bolt_server_stats* out);
int bolt_server_reset_stats(bolt_server* srv);

/* Stops the loop, waits for the device and frees every map of the server.
 * Requests still pending are abandoned.  NULL is a no-op. */
int bolt_server_destroy(bolt_server* srv);

/* ---------------------------------------------------------------------
 * Autotuning of the network schedules.
 *
 * Per array-length class 2^L (and device), the sort's tile (2^11, 2^12 or
 * 2^13 elements; the last runs in registers), the strides fused per global
 * sort pass (1..6) and the stages fused per global expansion pass (1..4).
 * Defaults: 13, 4, 4.  No choice changes any result, and every network's
 * memory accesses still depend on the array length alone; only speed
 * differs.  The table is per process and device.
 * --------------------------------------------------------------------- */

typedef struct {
  uint32_t log2_n;             /* the length class */
  uint32_t sort_tile_log;      /* 11..13 */
  uint32_t sort_pass_strides;  /* 1..6 */
  uint32_t expand_pass_stages; /* 1..4 */
  float sort_ms, expand_ms;    /* measured time of the chosen schedules */
} bolt_tune_entry;

/* Tunes the classes 2^14 .. 2^ceil(log2 n_max) (at most 2^28) on the
 * current device by timing every candidate on scratch arrays (it allocates
 * about 24 n_max bytes while it runs and synchronises the stream).  With a
 * cache_path: a cache file written earlier for this device is loaded
 * instead of tuning; otherwise the results are written there. */
int bolt_autotune(uint64_t n_max, const char* cache_path, void* hip_stream);

/* Reads the tuned entries of the current device (*n = how many there are). */
int bolt_tune_get(bolt_tune_entry* host_out, uint32_t cap, uint32_t* n);

/* Sets entries by hand (for example to test every schedule), and resets
 * the current device's table to the defaults. */
int bolt_tune_set(const bolt_tune_entry* host_in, uint32_t n);
int bolt_tune_reset(void);

/* ---------------------------------------------------------------------
 * Sealed commands and responses (BOLT_F_SEAL_CMDS).  The user's commands
 * reach the map encrypted and its responses leave encrypted, so the host
 * that relays them sees only their number and sizes (Sec. 3, threat model;
 * Sec. 5.1, the decode module opens commands and the response module seals
 * results).  Every command and every response is its own fixed-length
 * ChaCha20-Poly1305 (RFC 8439) record under the session key:
 *   command i of request seq   plain  LE64(op) || LE64(key) || value[vs]
 *                              nonce  LE32(i) || LE64(seq)
 *   its response               plain  LE64(status) || value[vs]
 *                              nonce  LE32(i | 2^31) || LE64(seq)
 *   both                       associated data LE64(q), q = the request's commands
 *   record                     cipher text || 16-byte tag
 * A command record is 32 + vs bytes, a response record 24 + vs.  Requests
 * of a map are numbered 1, 2, ... in the order the map runs them (the count
 * lives in device memory), so a replayed, reordered, truncated or changed
 * request fails its tags: it is then rejected whole (nothing changes, every
 * response status 0xFF) and the map is poisoned with BOLT_ETAMPER.
 * --------------------------------------------------------------------- */

/* Runs one sealed request of q commands (1..BOLT_MAX_BATCH): d_req holds q
 * command records, d_resp receives q response records (device memory,
 * caller-owned).  Stream-ordered like bolt_access_batch. */
int bolt_access_sealed(bolt_map* m, const void* d_req, uint32_t q, void* d_resp, void* hip_stream);

/* Client side (host memory, no device work): seals q commands as request
 * number seq into q command records, and opens q response records of
 * request seq (BOLT_ETAMPER if any fails its tag; its fields are then
 * zero).  value_bytes is the map's vs. */
int bolt_seal_requests(const uint8_t* session_key, uint64_t seq, uint32_t q, uint32_t value_bytes,
                       const uint8_t* ops, const uint64_t* keys, const void* vals, void* out_records);
int bolt_open_responses(const uint8_t* session_key, uint64_t seq, uint32_t q, uint32_t value_bytes,
                        const void* records, uint8_t* status, void* vals);

/* ---------------------------------------------------------------------
 * Device primitives of the path, exported so each can be checked alone.
 * --------------------------------------------------------------------- */

/* d_out[4 * i .. 4 * i + 3] = BLAKE2s-256 keyed with host_key[32] of the
 * nine bytes (domain, LE64(d_x[i])), as four little-endian 64-bit words:
 * the PRF that stands in for the key hash of Sec. 5.1 step 3 and for
 * random_remap of Alg. 1.  n may be 0. */
int bolt_prf(const uint8_t* host_key, uint8_t domain, const uint64_t* d_x, uint64_t n, uint64_t* d_out,
             void* hip_stream);

/* Sorts d_data[n] ascending in place with the bitonic sorting network used
 * by the build (n must be a power of two, 1 <= n <= 2^31).  The sequence of
 * memory accesses depends on n only. */
int bolt_sort_u64(uint64_t* d_data, uint64_t n, void* hip_stream);

/* Expansion network used by the build: d_elems[m] holds elements at
 * positions 0..n-1 as (target << 32 | payload) with strictly increasing
 * targets >= their position, and 0xFFFFFFFFFFFFFFFF from n on.  On return each
 * element sits at its target and every other position holds all ones.
 * d_tmp[m] is scratch.  Results are undefined if the targets break the rule. */
int bolt_expand_u64(uint64_t* d_elems, uint64_t* d_tmp, uint64_t m, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * expansion of bolt_expand_u64 without the d_tmp argument.  Its scratch is
 * a static device array of BOLT_NOALLOC_EXPAND_MAX elements (16 MiB) that
 * each GPU the library runs on holds until the process ends; the call
 * itself allocates and frees nothing.  m > BOLT_NOALLOC_EXPAND_MAX (or
 * m == 0, or a null d_elems) returns BOLT_EINVAL.  All calls on one GPU
 * share that GPU's scratch: calls ordered on one stream are safe, calls
 * that overlap on one GPU (different streams, several threads) race. */
#define BOLT_NOALLOC_EXPAND_MAX (1ull << 21)
int bolt_expand_u64_noalloc(uint64_t* d_elems, uint64_t m, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* BOLT_H */
