// Host-side state of one map and the launchers of its kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/bolt.h"
#include "bolt_dev.h"

namespace bolt {

// Scratch of one access batch, sized for BOLT_MAX_BATCH commands.
struct BatchScratch {
  uint32_t* leader;   // [Q] index of the first command with the same key
  uint32_t* prevw;    // [Q] last PUT/DEL of the same key before this command, or kNone
  uint32_t* lastw;    // [Q] (leaders) last PUT/DEL of the key in the batch, or kNone
  uint32_t* hit;      // [Q] (leaders) key found in the position map
  uint32_t* hrow;     // [Q] (leaders) its row
  uint32_t* hslot;    // [Q] (leaders) its slot in the row
  uint32_t* found;    // [Q] (leaders) item found in one of the two bins
  uint8_t* fval;      // [Q * vs] (leaders) the value found
  uint2* rpair;       // [Q] remap pair R(s) of each command
  uint32_t* cand_bin; // [3Q] bin each write-back candidate slot would rewrite, or kNone
  uint8_t* stage;     // [2Q * page_bytes] copies of the observable pages read
  uint8_t* outbox;    // [2][2Q * page_bytes] observable pages rebuilt by the write-back, by slot; a batch uses
                      // half (epoch & 1), so it rebuilds while the previous batch's half is still being sent
  uint32_t* ship_page;  // [2][2Q] observable page each write-back slot sends to the store, or kNone
  uint32_t* fin;      // [Q] (leaders) bit 0 present at the end, bit 1 found in the map
  uint32_t* chosen;   // [Q] (leaders placed) bin chosen by P2C
  uint32_t* rowsel;   // [Q] (keys inserted) position-map row chosen
  uint32_t* freed;    // [256] stash entries freed this batch, in buckets
  uint2* fpair;       // [Q] fetch pair F(s) of each command
  uint4* rows;        // [Q] position-map rows of each command's key
  uint32_t* rfree;    // BOLT_F_DECOMPOSED: [3Q][2Z] pool entries each rebuild slot returns to the ring
  uint8_t* rfree_n;   // BOLT_F_DECOMPOSED: [3Q] how many (bytes: at most 2Z <= 124)
};

struct TraceSeg {
  uint32_t batch;
  uint64_t offset;  // first word in the device log
  uint64_t reads;   // read words (2q), 0 for the build
  uint64_t writes;  // write words (2q for a batch, M for the build)
};

// Kernel classes timed with HIP events when a map has BOLT_F_TIMING.
enum KernelId {
  kkSortTile, kkSortGlobal, kkSortMerge, kkPairs, kkP2C, kkScan, kkExpand, kkWriteout, kkPmBuild, kkDupcheck,
  kkBuildMisc, kkAccDedup, kkAccFetch, kkAccResolve, kkAccRemap, kkAccCompose, kkAccShip, kkAccMisc, kkAccSolo, kkCount
};
extern const char* const kKernelNames[kkCount];

// Records a pair of events around each timed launch on its stream; the
// elapsed times are summed when read.  Events are recycled.
struct KernelTimer {
  struct Rec {
    int id;
    hipEvent_t a, b;
  };
  std::vector<hipEvent_t> pool;
  std::vector<Rec> recs;
  double total_ms[kkCount] = {};
  uint64_t launches[kkCount] = {};
  int cur = -1;
  hipEvent_t cur_a = nullptr;
  hipEvent_t take();
  void begin(int id, hipStream_t st);
  void end(hipStream_t st);
  int collect();  // after the stream is synchronised
  void reset();
  ~KernelTimer();
};

// Brackets launches with timer events when a timer is given.
struct TimedScope {
  KernelTimer* t;
  hipStream_t st;
  TimedScope(KernelTimer* t_, int id, hipStream_t s) : t(t_), st(s) {
    if (t) t->begin(id, st);
  }
  ~TimedScope() {
    if (t) t->end(st);
  }
};

struct Sizes {
  uint64_t cap, B, K, M, Z, W, d, R, page_bytes, stash_bound, P, BZ, PW, lmax, hbm_bound;
  uint32_t vs;
};

}  // namespace bolt

struct bolt_map {
  bolt_params p;
  bolt::Sizes s;
  int device;
  // persistent device state
  bolt::Ctl* ctl;
  uint8_t* obs;       // M pages (device pointer; maps pinned host memory in host mode)
  uint8_t* obs_host;  // host pointer of the pinned store, or null
  uint8_t* hbm;       // K HBM bins (null in a decomposed store)
  uint32_t* ring;     // BOLT_F_DECOMPOSED: [P] the value pool's free-address ring, else null
  uint32_t* load;     // [B]
  uint32_t* load0;    // [B] the loads a batch's placement starts from (removals in, adds not)
  uint64_t* pm_key;   // [R * W]
  uint2* pm_pair;     // [R * W]
  uint32_t* pm_mask;  // [R] used slots
  uint64_t* st_key;   // [P] stash pool
  uint8_t* st_val;    // [P * vs]
  uint32_t* st_dest;  // [P] destination bin
  uint32_t* st_dead;  // [P] removed by an access of this batch
  uint64_t* st_used;  // [ceil(P / 64)] pool bitmap, 1 = in use
  uint32_t* rev_cnt;  // [B] stash entries listed per bin
  uint32_t* rev_idx;  // [B * 2Z]
  uint64_t* claim;    // [B] write-back election, tagged with the batch epoch
  uint64_t* rmask;    // [B] page slots removed in this batch
  uint32_t* tlog;     // trace log (BOLT_F_TRACE)
  uint64_t tlog_cap, tlog_used;
  bool tlog_lost;
  std::vector<bolt::TraceSeg> segs;
  bolt::BatchScratch bs;
  uint8_t* get_ops;   // [Q] all BOLT_OP_GET (bolt_get_batch)
  uint8_t* put_ops;   // [Q] all BOLT_OP_PUT (bolt_put_batch)
  uint8_t* discard;   // [2Q * vs] unused inputs / outputs of those wrappers
  // BOLT_F_SEAL_CMDS: the opened commands and the plain responses of a
  // sealed request (device memory only)
  uint8_t* sc_ops;    // [Q]
  uint64_t* sc_keys;  // [Q]
  uint8_t* sc_vin;    // [Q * vs]
  uint8_t* sc_vout;   // [Q * vs]
  uint8_t* sc_st;     // [Q]
  std::vector<void*> allocs;  // every hipMalloc of this map
  bool built, poisoned;
  int sticky;
  uint64_t batches;
  hipStream_t last_stream;
  bolt::KernelTimer* timer;  // BOLT_F_TIMING, else null
  // The build's position-map rounds run on `side`, forked from and joined
  // back to the caller's stream with the two events.
  hipStream_t side;
  hipEvent_t ev_fork, ev_join;
  // BOLT_F_GRAPHS: one access plan on the device, and the graph of the
  // access pipeline captured per batch-size class ceil(log2 q) = 0..13.
  void* gplan;
  hipGraphExec_t gexec[14];
  // BOLT_F_SEAL: tags beside the observable pages, write counts in HBM
  uint8_t* tags;    // [M * 16], observable (device address)
  uint64_t* pver;   // [M]
  // The write-back rebuilds a batch's observable pages in HBM (the outbox);
  // they go to the store during the next batch's fetch, whose workgroups
  // read pages over the link while these write (both directions at once),
  // or when bolt_flush or a reader of the store asks.  wslot[p] holds
  // (batch epoch << 32 | outbox slot) of the last rebuild of page p, so that
  // fetch takes such a page from the outbox (it still reads the store's
  // copy, for the same trace).
  uint64_t* wslot;  // [M]
  uint32_t ship_q;     // commands of the batch whose pages are still to be sent, 0 = none
  uint32_t ship_from;  // its outbox slots [ship_from, 2 ship_q) are still to be sent
  uint32_t ship_half;  // its half of the outbox (its epoch & 1)
  bool ov_off;        // next batch: no outbox pages (the store was changed from the host)
};

namespace bolt {

void launch_prf_key_setup(Ctl* ctl, const uint8_t key[32], hipStream_t st);
void launch_prf_array(const Ctl* ctl, uint32_t domain, const uint64_t* x, uint64_t n, uint64_t* out, hipStream_t st);
// One array of a many-array network launch: data, scratch of the same
// length (expansion only), and the length (a power of two for the sort).
struct NetSeg {
  uint64_t* a;
  uint64_t* b;
  uint64_t n;
};

// Schedule of the network kernels for arrays of length class 2^log2n:
// sort tile 2^sort_tile_log (11..13), strides per global sort pass
// (1..4), stages per global expansion pass (1..4).  Defaults 13 / 4 / 4;
// bolt_autotune measures and replaces them.  No choice changes a result.
struct NetTune {
  uint32_t sort_tile_log, sort_fmax, exp_fmax;
};
NetTune net_tune(uint32_t log2n);

void launch_bitonic_sort(uint64_t* a, uint64_t n, hipStream_t st, KernelTimer* tm = nullptr);
void launch_bitonic_sort_with(uint64_t* a, uint64_t n, hipStream_t st, uint32_t tile_log, uint32_t fmax);
uint64_t* launch_expand_with(uint64_t* a, uint64_t* tmp, uint64_t m, hipStream_t st, uint32_t fmax);
void launch_bitonic_sort_many(const NetSeg* segs, uint32_t count, uint64_t nmax, hipStream_t st);
void launch_expand(uint64_t* a, uint64_t* tmp, uint64_t m, hipStream_t st, KernelTimer* tm = nullptr);
// As launch_expand without the final copy: returns the buffer holding the result.
uint64_t* launch_expand_inplace(uint64_t* a, uint64_t* tmp, uint64_t m, hipStream_t st, KernelTimer* tm = nullptr);
// Returns true when every array's result ended in its scratch (b).
bool launch_expand_many(const NetSeg* segs, uint32_t count, uint64_t mmax, hipStream_t st);

void launch_map_init(bolt_map* m, hipStream_t st);
int run_build(bolt_map* m, const uint64_t* keys, const void* vals, uint64_t n, hipStream_t st);
int run_build_many(bolt_map* const* maps, const uint64_t* const* keys, const void* const* vals, const uint64_t* n,
                   uint32_t count, hipStream_t st);
int run_access(bolt_map* m, const uint8_t* ops, const uint64_t* keys, const void* vals_in, void* vals_out,
               uint8_t* status, uint32_t q, hipStream_t st);
// defer_pages: large batches on pinned stores rebuild their pages into the
// outbox, sent by each map's next batch (or a flush); else the rebuild
// writes them.  The pages pending from each map's previous batch always go
// out from this launch's fetch.
int run_access_many(bolt_map* const* maps, const bolt_batch* batches, uint32_t count, hipStream_t st,
                    bool defer_pages);
// bolt_access_many's checks and dispatch, with the page-send choice above.
int access_many(bolt_map* const* maps, const bolt_batch* batches, uint32_t count, void* hip_stream,
                bool defer_pages);
// Sends the rebuilt pages of the map's last batch to the store, if any.
int flush_ship(bolt_map* m, hipStream_t st);
// Sealed requests (k_record.hip): commands t of a call (requests starting
// at tab[r], nreq of them; tab null = one request of q) opened into plain
// arrays, and responses sealed from them; the seal also advances the
// map's request count past the call.
void launch_rec_open(bolt_map* m, const void* recs, uint32_t q, const uint32_t* tab, uint32_t nreq, uint8_t* ops,
                     uint64_t* keys, void* vals, hipStream_t st);
void launch_rec_seal(bolt_map* m, void* out, uint32_t q, const uint32_t* tab, uint32_t nreq, const uint8_t* status,
                     const void* vals, hipStream_t st);

}  // namespace bolt
