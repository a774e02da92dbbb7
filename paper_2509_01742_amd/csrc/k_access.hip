// Batched oblivious access (Alg. 1 per command, in the module order of
// Sec. 5.1): decode, key search, value access, remap + eviction, response.
//
// One batch of q commands runs as a handful of kernels on one stream:
//   dedup     one workgroup sorts (key, index) (registers, wave shuffles,
//             LDS); leader = first command of each key; for every command
//             the last PUT/DEL of its key before it
//   fetch     one wave per command: tape T(s) -> fetch pair F(s) and remap
//             pair R(s); leaders look their key up in the position map (d
//             rows); read both bins whole (observable pages are copied to
//             a staging area); the leader of a mapped key finds and removes
//             its item (page slot or stash entry); elect one writer per bin
//   resolve   responses of every command in index order (sequential
//             semantics of the batch); final state of every key
//   remap     keys present at the end get R(s) and P2C over the
//             post-removal loads, in rounds of ceil(B/16) keys; the item goes
//             to the stash pool, listed under its bin; position-map
//             updates, deletes, then inserts in rounds of ceil(R/16).  When
//             the batch fits one round of each (large maps) this runs
//             thread-per-command across the chip (resolve decides, place
//             applies, finish inserts); otherwise one workgroup runs the
//             rounds in order
//   writeback one wave per candidate bin: the elected writer rebuilds the
//             bin as survivors + every live stash item listed for it,
//             canonical order, and writes it whole (observable pages once
//             each); the entries listed are freed
//   finish    position-map inserts (one-round case), counters, stash bound
#include <string.h>

#include <vector>

#include <mutex>

#include "bolt_impl.h"
#include "seal_dev.h"

namespace bolt {

// The send of a batch's rebuilt observable pages to the store.
struct ShipArgs {
  const Ctl* ctl;
  uint32_t lo, hi;  // the slots [lo, hi) of the batch's outbox
  uint64_t pw;
  const uint32_t* ship_page;
  const uint64_t* outbox;
  uint64_t* obs;
  uint64_t* tags;  // BOLT_F_SEAL: [M][2] page tags, else null
  uint64_t* pver;  // BOLT_F_SEAL: [M] page write counts
};

struct GroupArgs {
  const uint8_t* ops;
  const uint64_t* keys;
  uint32_t q, epoch;
  uint64_t B, R;
  Ctl* ctl;
  uint32_t* leader;
  uint32_t* prevw;
  uint32_t* lastw;
  uint2* fpair;
  uint2* rpair;
  uint4* rows;
  ShipArgs ship;  // a slice of the previous batch's send, by the first ship_blocks workgroups
  uint32_t ship_blocks;
};


struct FetchArgs {
  const Ctl* ctl;
  const uint8_t* ops;
  const uint64_t* keys;
  const uint32_t* leader;
  const uint2* fpair;
  const uint4* rows;
  uint32_t q, epoch;
  uint64_t B, K, R;
  uint32_t Z, W, d, vw;
  uint64_t pw;  // page words
  const uint64_t* pm_key;
  const uint2* pm_pair;
  const uint32_t* pm_mask;
  const uint64_t* obs;
  const uint64_t* hbm;
  const uint32_t* rev_cnt;
  const uint32_t* rev_idx;
  const uint64_t* st_key;
  const uint64_t* st_val;
  uint32_t* st_dead;
  uint32_t* load;
  uint32_t* load0;  // the loads placement starts from: removals go to both
  uint64_t* claim;
  uint64_t* rmask;
  uint64_t* stage;
  uint32_t* cand_bin;
  uint32_t* hit;
  uint32_t* hrow;
  uint32_t* hslot;
  uint32_t* found;
  uint64_t* fval;
  uint2* rpair;
  uint32_t* tlog_r;  // [2q] or null
  Ctl* ctlw;
  const uint64_t* tags;  // BOLT_F_SEAL: [M][2] page tags, else null
  const uint64_t* pver;  // BOLT_F_SEAL: [M] page write counts
  const uint64_t* wslot;   // [M] last rebuild of each page: epoch << 32 | outbox slot
  const uint64_t* outbox;  // [2Q][pw] the previous batch's rebuilt pages
  uint32_t ov_epoch;       // epoch whose rebuilt pages the outbox holds, 0 = none
  ShipArgs ship;           // a slice of the previous batch's send ...
  uint32_t ship_blocks;    // ... by the first ship_blocks workgroups
  uint32_t pre_host;       // 1: observable pages are read ahead too (device store)
  uint32_t decomp;         // BOLT_F_DECOMPOSED: an HBM bin is only its list (no page)
  // one-round batches: a leader whose key is mapped and absent at the end
  // of the batch deletes its map entry here (its last PUT/DEL, else whether
  // it was found, decides), so that every delete is in before placement
  uint32_t fast;
  const uint32_t* lastw;
  uint32_t* pm_mask_w;
};

struct ResolveArgs {
  Ctl* ctl;
  const uint8_t* ops;
  const uint64_t* vals_in;
  const uint32_t* leader;
  const uint32_t* prevw;
  const uint32_t* lastw;
  const uint32_t* hit;
  const uint32_t* hrow;
  const uint32_t* hslot;
  const uint32_t* found;
  const uint64_t* fval;
  const uint2* rpair;
  const uint32_t* load;  // the loads as placement began
  uint32_t q, vw, fast, epoch;
  uint64_t* vals_out;
  uint8_t* status;
  uint32_t* fin;
  uint32_t* chosen;
  ShipArgs ship;  // a slice of the previous batch's send, by the first ship_blocks workgroups
  uint32_t ship_blocks;
};

struct PlaceArgs {
  // The batch takes the several-round path: k_acc_remap chose the bins and
  // added the loads (rounds of ceil(B/16)), and puts the inserts in their
  // rows (rounds of ceil(R/16)) after this kernel.
  uint32_t several;
  Ctl* ctl;
  const uint64_t* keys;
  const uint64_t* vals_in;
  const uint32_t* leader;
  const uint32_t* lastw;
  const uint32_t* fin;
  const uint32_t* chosen;
  const uint32_t* hrow;
  const uint32_t* hslot;
  const uint64_t* fval;
  const uint2* rpair;
  uint32_t q, epoch, Z, W, d, vw;
  uint64_t K, R, PW;
  uint32_t* load;
  uint64_t* st_used;
  uint64_t* st_key;
  uint64_t* st_val;
  uint32_t* st_dest;
  uint32_t* st_dead;
  uint32_t* rev_cnt;
  uint32_t* rev_idx;
  uint64_t* claim;
  uint32_t* cand_bin;
  uint2* pm_pair;
  const uint32_t* pm_mask;
  uint32_t* rowsel;
  const uint4* rows;  // [Q] position-map rows of each command's key (from the dedup kernel)
  ShipArgs ship;  // a slice of the previous batch's send, by the first ship_blocks workgroups
  uint32_t ship_blocks;
  uint32_t decomp;  // BOLT_F_DECOMPOSED: entries come from the free-address ring
  uint32_t* ring;
  uint64_t P;
};

struct RemapArgs {
  uint32_t enabled;  // this map's batch takes the several-round path
  Ctl* ctl;
  uint32_t* chosen;  // [Q] each placed key's bin, for k_acc_place
  const uint64_t* keys;
  const uint64_t* vals_in;
  const uint32_t* leader;
  const uint32_t* lastw;
  const uint32_t* fin;
  const uint32_t* hrow;
  const uint32_t* hslot;
  const uint64_t* fval;
  const uint2* rpair;
  uint32_t q, epoch, Z, W, d, vw;
  uint64_t B, K, R, PW;
  uint32_t* load;
  uint64_t* st_used;
  uint64_t* st_key;
  uint64_t* st_val;
  uint32_t* st_dest;
  uint32_t* st_dead;
  uint32_t* rev_cnt;
  uint32_t* rev_idx;
  uint64_t* claim;
  uint32_t* cand_bin;
  uint64_t* pm_key;
  uint2* pm_pair;
  uint32_t* pm_mask;
  const uint4* rows;  // [Q] position-map rows of each command's key
  uint32_t decomp;    // BOLT_F_DECOMPOSED: entries come from the free-address ring
  uint32_t* ring;
  uint64_t P;
};

struct WbArgs {
  Ctl* ctl;
  uint32_t q, epoch, Z, vw;
  uint64_t K, pw;
  const uint32_t* cand_bin;
  const uint64_t* claim;
  uint64_t* rmask;
  const uint64_t* stage;
  uint64_t* hbm;
  uint32_t* rev_cnt;
  uint32_t* rev_idx;
  const uint64_t* st_key;
  const uint64_t* st_val;
  uint32_t* st_dead;
  uint64_t* st_used;
  uint32_t* freed;      // [kFreeBuckets] entries freed, summed by finish
  uint32_t* tlog_w;     // [3q] or null
  uint64_t* outbox;     // [2Q][pw] rebuilt observable pages, by slot (this batch's half)
  uint32_t* ship_page;  // [2Q] page each slot sends, or kNone (this batch's half)
  uint64_t* wslot;      // [M]
  uint32_t direct;      // 1: write observable pages to the store here (no send)
  uint64_t* obs;        // direct: the store
  uint64_t* tags;       // direct, BOLT_F_SEAL: [M][2] page tags, else null
  uint64_t* pver;       // direct, BOLT_F_SEAL: [M] page write counts
  ShipArgs ship;  // a slice of the previous batch's send, by the first ship_blocks workgroups
  uint32_t ship_blocks;
  uint32_t decomp;  // BOLT_F_DECOMPOSED: HBM bins keep their items listed; frees are staged for the ring
  uint32_t* rfree;    // [3Q][2Z] entries each rebuild slot returns to the ring
  uint8_t* rfree_n;   // [3Q] how many (at most 2Z <= 124)
  // each placed key's bin, whose final load the next batch's placement starts from
  const uint32_t* leader;
  const uint32_t* fin;
  const uint32_t* chosen;
  const uint32_t* load;
  uint32_t* load0;
};


struct FinishArgs {
  Ctl* ctl;
  uint32_t q, W, epoch;
  uint64_t cap, stash_bound, hbm_bound;
  const uint32_t* rowsel;
  const uint64_t* keys;
  const uint2* rpair;
  uint32_t* freed;
  uint64_t* pm_key;
  uint2* pm_pair;
  uint32_t* pm_mask;
  ShipArgs ship;  // a slice of the previous batch's send, by the first ship_blocks workgroups
  uint32_t ship_blocks;
  uint32_t decomp;          // BOLT_F_DECOMPOSED: the finish appends the staged frees to the ring
  uint32_t Z2;              // 2Z, the stride of rfree
  uint32_t* ring;
  uint64_t P;
  const uint32_t* rfree;    // [3Q][2Z]
  const uint8_t* rfree_n;   // [3Q], 16-byte aligned
};

// Every kernel argument of one map's batch.  A multi-map launch reads the
// plan of map blockIdx.y from a device table; a single-map launch passes
// the argument block by value.
struct AccessPlan {
  GroupArgs gr;
  FetchArgs fa;
  ResolveArgs rv;
  PlaceArgs pa;
  RemapArgs ra;
  WbArgs wa;
  FinishArgs fn;
  uint32_t q, fast;
  uint64_t wb_lds;     // dynamic LDS of the write-back
  uint64_t fetch_lds;  // dynamic LDS of the fetch (sealed maps; a send it carries uses the same)
};

#define BOLT_PICK(T, field) const T& a = MULTI ? tab[blockIdx.y].field : a1

constexpr uint32_t kDedupNT = 1024;
constexpr uint32_t kDedupPer = kMaxBatch / kDedupNT;  // 8 sorted positions per thread

__device__ __forceinline__ uint64_t claim_tag(uint32_t epoch, uint32_t slot) {
  return ((uint64_t)epoch << 32) | (uint64_t)(0xFFFFFFFFu - slot);
}

__device__ __forceinline__ uint32_t wave_incl_max(uint32_t x) {
  const uint32_t lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    uint32_t y = __shfl_up(x, off, 64);
    if (lane >= (uint32_t)off) x = x > y ? x : y;
  }
  return x;
}

__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t x) {
  const uint32_t lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    uint32_t y = __shfl_up(x, off, 64);
    if (lane >= (uint32_t)off) x += y;
  }
  return x;
}

// Position of the k-th (from 0) set bit of x; k < popcount(x).
__device__ __forceinline__ uint32_t select_set_bit(uint64_t x, uint32_t k) {
  uint32_t pos = 0;
#pragma unroll
  for (uint32_t half = 32; half >= 1; half >>= 1) {
    const uint32_t c = (uint32_t)__popcll(x & ((1ull << half) - 1));
    if (k >= c) {
      k -= c;
      x >>= half;
      pos += half;
    }
  }
  return pos;
}

// Stash-pool entries for the lanes of a wave that want one (every lane of
// the wave calls this).  The wave reads a window of up to 64 consecutive
// bitmap words at once, starting at `start`, hands the lanes that still need
// an entry the free bits of the window in order, and each word's lane sets
// the bits it handed out with one atomicOr: one atomic per word for the
// wave, where an atomic per lane would queue dozens on the few lines of a
// small map's bitmap.  A lane whose bit another wave took first tries again;
// an empty window moves the wave on.  kNone for a lane only when every word
// was seen full in a row (no entry is freed while entries are taken).  Each
// pass takes a bit or moves on, so the loop ends within 65 * nwords + 64.
__device__ __forceinline__ uint32_t pool_alloc_wave(uint64_t* used, uint64_t nwords, uint64_t start, bool want) {
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t below = (1ull << lane) - 1;
  uint64_t need = __ballot(want);
  uint32_t got = kNone;
  const uint32_t span = nwords < 64 ? (uint32_t)nwords : 64u;
  uint64_t w0 = start % nwords, empty = 0;
  for (uint64_t it = 0; need && it < 65 * nwords + 64; ++it) {
    const uint64_t w = (w0 + lane) % nwords;
    const uint64_t cur = lane < span ? __hip_atomic_load(&used[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : ~0ull;
    const uint32_t fc = (uint32_t)__popcll(~cur);
    const uint32_t incl = wave_incl_sum(fc), excl = incl - fc;
    const uint32_t total = (uint32_t)__shfl((int)incl, 63, 64);
    if (total == 0) {  // the same for the whole wave
      w0 = (w0 + span) % nwords;
      empty += span;
      if (empty >= nwords) break;
      continue;
    }
    empty = 0;
    // the pending lanes' ranks 0 .. min(npend, total) - 1 go to the words
    // in order, the lowest free bits of each word first
    const uint32_t npend = (uint32_t)__popcll(need);
    const uint32_t g = npend > excl ? (npend - excl < fc ? npend - excl : fc) : 0;
    uint64_t old = 0;
    if (g) {
      const uint32_t top = select_set_bit(~cur, g - 1);
      const uint64_t mask = ~cur & (top == 63 ? ~0ull : ((2ull << top) - 1));
      old = atomicOr((unsigned long long*)&used[w], (unsigned long long)mask);
    }
    const uint32_t r = (uint32_t)__popcll(need & below);
    uint32_t j = 0;  // the last lane whose word's ranks start at or below r
#pragma unroll
    for (uint32_t step = 32; step >= 1; step >>= 1) {
      const uint32_t c = j + step;
      const uint32_t ec = (uint32_t)__shfl((int)excl, (int)(c < 64 ? c : 63), 64);
      if (c < 64 && ec <= r) j = c;
    }
    const uint64_t cur_j = __shfl(cur, (int)j, 64), old_j = __shfl(old, (int)j, 64), w_j = __shfl(w, (int)j, 64);
    const uint32_t excl_j = (uint32_t)__shfl((int)excl, (int)j, 64);
    if (((need >> lane) & 1) && r < npend && r < total) {
      const uint32_t pos = select_set_bit(~cur_j, r - excl_j);
      if (!((old_j >> pos) & 1)) got = (uint32_t)(w_j * 64 + pos);
    }
    need &= ~__ballot(got != kNone);
  }
  return got;
}

// Block-wide exclusive scans over one value per thread (NT threads).
template <int NT, bool MAX>
__device__ uint32_t block_excl(uint32_t x, uint32_t* total) {
  __shared__ uint32_t ws[NT / 64];
  const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint32_t inc = MAX ? wave_incl_max(x) : wave_incl_sum(x);
  if (lane == 63) ws[wid] = inc;
  __syncthreads();
  if (wid == 0) {
    uint32_t v = lane < NT / 64 ? ws[lane] : 0;
    uint32_t vi = MAX ? wave_incl_max(v) : wave_incl_sum(v);
    uint32_t ex = __shfl_up(vi, 1, 64);
    if (lane == 0) ex = 0;
    if (lane < NT / 64) ws[lane] = ex;
    if (lane == NT / 64 - 1) *total = vi;
  }
  __syncthreads();
  uint32_t before = ws[wid];
  uint32_t wex = __shfl_up(inc, 1, 64);
  if (lane == 0) wex = 0;
  uint32_t r = MAX ? (before > wex ? before : wex) : before + wex;
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------------------
// dedup + fold structure (one workgroup)
// ---------------------------------------------------------------------------

// (key, index) strictly before (key', index')
__device__ __forceinline__ bool kv_less(uint64_t ka, uint32_t ia, uint64_t kb, uint32_t ib) {
  return ka < kb || (ka == kb && ia < ib);
}

// Compare-exchange of the pairs (e, e + J) held by one thread (J < 8 known at
// compile time, so the arrays stay in registers).
template <uint32_t J>
__device__ __forceinline__ void dedup_reg_stage(uint64_t k[kDedupPer], uint32_t x[kDedupPer], uint32_t base,
                                                uint32_t kk) {
#pragma unroll
  for (uint32_t e = 0; e < kDedupPer; ++e) {
    if (e & J) continue;
    const uint32_t e2 = e + J;
    const bool asc = ((base + e) & kk) == 0;
    const bool lt = kv_less(k[e2], x[e2], k[e], x[e]);
    const bool gt = kv_less(k[e], x[e], k[e2], x[e2]);
    if (asc ? lt : gt) {
      const uint64_t tk = k[e];
      k[e] = k[e2];
      k[e2] = tk;
      const uint32_t tx = x[e];
      x[e] = x[e2];
      x[e2] = tx;
    }
  }
}

// Bitonic sort of the (key, index) pairs: thread t holds positions 8t..8t+7.
// Strides 1..4 run inside a thread, strides 8..256 between lanes of a wave
// (shuffles), strides 512 and up through LDS.
__device__ __forceinline__ void dedup_sort(uint64_t k[kDedupPer], uint32_t x[kDedupPer], uint32_t npad,
                                           uint64_t* skey, uint32_t* sidx) {
  const uint32_t base = threadIdx.x * kDedupPer;
  // A wave whose positions all lie at or past npad holds only padding, and
  // no stage of a network of size npad pairs it with a real position: it
  // skips the register and shuffle stages (it still meets every barrier).
  const bool busy = (threadIdx.x & ~63u) * kDedupPer < npad;
  for (uint32_t kk = 2; kk <= npad; kk <<= 1) {
    for (uint32_t j = kk >> 1; j > 0; j >>= 1) {
      if (!busy && j < 64 * kDedupPer) continue;
      if (j < kDedupPer) {
        if (j == 4) dedup_reg_stage<4>(k, x, base, kk);
        else if (j == 2) dedup_reg_stage<2>(k, x, base, kk);
        else dedup_reg_stage<1>(k, x, base, kk);
      } else if (j < 64 * kDedupPer) {
        const int d = (int)(j / kDedupPer);
#pragma unroll
        for (uint32_t e = 0; e < kDedupPer; ++e) {
          const uint64_t ok = __shfl_xor(k[e], d, 64);
          const uint32_t ox = __shfl_xor(x[e], d, 64);
          const uint32_t p = base + e;
          const bool keep_min = ((p & j) == 0) == ((p & kk) == 0);
          const bool take = keep_min ? kv_less(ok, ox, k[e], x[e]) : kv_less(k[e], x[e], ok, ox);
          if (take) {
            k[e] = ok;
            x[e] = ox;
          }
        }
      } else {  // positions past npad (no LDS for them) are padding, paired with padding
        if (base < npad) {
#pragma unroll
          for (uint32_t e = 0; e < kDedupPer; ++e) {
            skey[base + e] = k[e];
            sidx[base + e] = x[e];
          }
        }
        __syncthreads();
        if (base < npad) {
#pragma unroll
          for (uint32_t e = 0; e < kDedupPer; ++e) {
            const uint32_t p = base + e;
            const uint64_t ok = skey[p ^ j];
            const uint32_t ox = sidx[p ^ j];
            const bool keep_min = ((p & j) == 0) == ((p & kk) == 0);
            const bool take = keep_min ? kv_less(ok, ox, k[e], x[e]) : kv_less(k[e], x[e], ok, ox);
            if (take) {
              k[e] = ok;
              x[e] = ox;
            }
          }
        }
        __syncthreads();
      }
    }
  }
  if (base < npad) {
#pragma unroll
    for (uint32_t e = 0; e < kDedupPer; ++e) {
      skey[base + e] = k[e];
      sidx[base + e] = x[e];
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// send of rebuilt observable pages
// ---------------------------------------------------------------------------

// The send of a batch's rebuilt observable pages to the store: wave `wave`
// of `waves` takes the slots lo + wave, lo + wave + waves, ... below hi.  Plain maps copy the
// page; sealed maps encrypt it in the wave's LDS page `pg` under the page's
// next write count, tag it, and write page and tag.
template <bool SEALED>
__device__ __forceinline__ void ship_slots(const ShipArgs& a, uint32_t wave, uint32_t waves, uint64_t* pg) {
  const uint32_t lane = threadIdx.x & 63;
  uint32_t key[8];
  if (SEALED) {
#pragma unroll
    for (int j = 0; j < 8; ++j) key[j] = a.ctl->skey[j];
  }
  for (uint32_t s = a.lo + wave; s < a.hi; s += waves) {
    const uint32_t page = a.ship_page[s];
    if (page == kNone) continue;  // whole wave
    const uint64_t* src = a.outbox + (uint64_t)s * a.pw;
    uint64_t* dst = a.obs + (uint64_t)page * a.pw;
    if (!SEALED) {
      for (uint64_t w = lane; w < a.pw; w += 64) dst[w] = src[w];
      continue;
    }
    for (uint64_t w = lane; w < a.pw; w += 64) pg[w] = src[w];
    const uint64_t ver = a.pver[page] + 1;
    uint32_t tag[4];
    seal_page(pg, (uint32_t)a.pw, key, page, ver, dst, tag);
    if (lane == 0) {
      a.tags[2 * (uint64_t)page] = (uint64_t)tag[0] | ((uint64_t)tag[1] << 32);
      a.tags[2 * (uint64_t)page + 1] = (uint64_t)tag[2] | ((uint64_t)tag[3] << 32);
      a.pver[page] = ver;
    }
    wave_sync();  // the wave's LDS page is reused by its next slot
  }
}

// Workgroups (of 4 waves) of a send of n slots: one per 4 slots, at most
// 256, so that the kernel it rides with keeps most of the device.
constexpr uint32_t kShipMaxBlocks = 256;
__host__ __device__ constexpr uint32_t ship_blocks_for(uint32_t n) {
  return (n + 3) / 4 < kShipMaxBlocks ? (n + 3) / 4 : kShipMaxBlocks;
}

// Workgroups [0, ship_blocks) of a kernel that carries a slice of a send
// (plain maps only: no LDS) do that and nothing else; true for them.
template <bool MULTI>
__device__ __forceinline__ bool carry_ship(const ShipArgs& sh, uint32_t ship_blocks) {
  if (MULTI || blockIdx.x >= ship_blocks) return false;
  const uint32_t wpb = blockDim.x >> 6;  // waves per workgroup
  ship_slots<false>(sh, blockIdx.x * wpb + (threadIdx.x >> 6), ship_blocks * wpb, nullptr);
  return true;
}

// A send on its own (bolt_flush, readers of the store, many-map calls).
__global__ __launch_bounds__(256) void k_acc_ship(ShipArgs a) {
  extern __shared__ uint64_t sdyn[];
  const uint32_t wv = threadIdx.x >> 6;
  if (a.tags)
    ship_slots<true>(a, blockIdx.x * 4 + wv, gridDim.x * 4, sdyn + (uint64_t)wv * a.pw);
  else
    ship_slots<false>(a, blockIdx.x * 4 + wv, gridDim.x * 4, nullptr);
}

// Commands are first split into kParts partitions by a hash of their key
// (all commands of a key land in one partition); each partition is then
// sorted and folded by its own workgroup.
constexpr uint32_t kParts = 64;

__device__ __forceinline__ uint64_t key_mix(uint64_t key) {
  uint64_t x = key;
  x ^= x >> 33;
  x *= 0xFF51AFD7ED558CCDull;
  x ^= x >> 33;
  return x;
}
__device__ __forceinline__ uint32_t part_of(uint64_t key) { return (uint32_t)(key_mix(key) >> 58); }  // kParts = 64

// Slots of the LDS hash table that folds a partition of up to kDedupNT
// commands (at most half full).
constexpr uint32_t kHashSlots = 2 * kDedupNT;

// Workgroups of the dedup kernel that compute PRFs, two per command: 256
// threads of each (one wave per SIMD: a PRF is a long run of dependent
// integer operations, and waves sharing a SIMD would queue behind each other).
constexpr uint32_t kPrfPerBlock = 256;
__host__ __device__ constexpr uint32_t group_prf_blocks(uint32_t q) { return (2 * q + kPrfPerBlock - 1) / kPrfPerBlock; }

// Entries of the dedup kernel's partition arrays for a batch of q commands
// (the sort of a large partition pads it to a power of two), and its bytes
// of dynamic LDS.
__host__ __device__ constexpr uint32_t group_lds_entries(uint32_t q) {
  uint32_t n = 64;
  while (n < q) n <<= 1;
  return n;
}
__host__ __device__ constexpr uint64_t group_lds_bytes(uint32_t q) { return 12ull * group_lds_entries(q); }

// PRF t of a batch, two per command i = t / 2: for even t the fetch pair
// F(s) and remap pair R(s) of tape step s, for odd t the key's position-map
// rows.
__device__ __forceinline__ void group_prf(const GroupArgs& a, uint32_t t) {
  const uint32_t i = t >> 1;
  uint32_t hk[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) hk[j] = a.ctl->hkey[j];
  uint64_t w[4];
  if ((t & 1) == 0) {
    prf4(hk, kDomTape, a.ctl->steps + i, w);
    uint32_t f1, f2, r1, r2;
    pair_of(w[0], w[1], a.B, f1, f2);
    pair_of(w[2], w[3], a.B, r1, r2);
    a.fpair[i] = make_uint2(f1, f2);
    a.rpair[i] = make_uint2(r1, r2);
  } else {
    prf4(hk, kDomRows, a.keys[i], w);
    a.rows[i] = make_uint4((uint32_t)__umul64hi(w[0], a.R), (uint32_t)__umul64hi(w[1], a.R),
                           (uint32_t)__umul64hi(w[2], a.R), (uint32_t)__umul64hi(w[3], a.R));
  }
}

// One workgroup per partition (kParts of them), then group_prf_blocks(q)
// workgroups for the PRF outputs, which run beside them.  A partition's
// workgroup picks the commands of its partition out of the whole batch (all
// commands of a key land in one partition) and derives for each command its
// leader (first command of its key), the last PUT/DEL of its key before it,
// and for each leader the last PUT/DEL of its key in the batch.  A batch
// with an op code above DEL is marked rejected.
template <bool MULTI>
__global__ __launch_bounds__(kDedupNT) void k_acc_group(GroupArgs a1, const AccessPlan* tab) {
  BOLT_PICK(GroupArgs, gr);
  const uint8_t* __restrict__ ops = a.ops;
  const uint64_t* __restrict__ keys = a.keys;
  const uint32_t qall = a.q;
  uint32_t* __restrict__ leader = a.leader;
  uint32_t* __restrict__ prevw = a.prevw;
  uint32_t* __restrict__ lastw = a.lastw;
  // the partition's (key, index << 2 | op) entries, in dynamic LDS sized for
  // the whole batch (a partition may hold every command)
  extern __shared__ uint64_t gdyn[];
  uint64_t* const skey = gdyn;
  uint32_t* const sidx = reinterpret_cast<uint32_t*>(gdyn + group_lds_entries(qall));
  __shared__ uint32_t tot;
  if (carry_ship<MULTI>(a.ship, a.ship_blocks)) return;
  const uint32_t part = blockIdx.x - (MULTI ? 0 : a.ship_blocks);
  const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (part >= kParts) {
    // The blocks past the partitions compute the PRF outputs, two per
    // command (thread t: PRF t): the fetch pair F(s) and remap pair R(s) of
    // tape step s, and the key's position-map rows.
    if (threadIdx.x >= kPrfPerBlock) return;
    const uint32_t t = (part - kParts) * kPrfPerBlock + threadIdx.x;
    if ((t >> 1) < qall) group_prf(a, t);
    return;
  }
  // This partition's commands, gathered in index order: every command's key
  // and op code loaded at once (one chunk of kDedupNT per register), a
  // ballot per wave and chunk, then the (chunk, wave) counts' prefix.
  constexpr uint32_t kChunks = kMaxBatch / kDedupNT;
  uint64_t ckey[kChunks];
  uint32_t cop[kChunks];
#pragma unroll
  for (uint32_t c = 0; c < kChunks; ++c) {
    const uint32_t i = c * kDedupNT + threadIdx.x;
    ckey[c] = i < qall ? keys[i] : 0;
    cop[c] = i < qall ? ops[i] : 0;
  }
  __shared__ uint32_t wcnt[kChunks][kDedupNT / 64];
  const uint32_t nch = (qall + kDedupNT - 1) / kDedupNT;
  uint64_t bal[kChunks];
  bool bad = false;
#pragma unroll
  for (uint32_t c = 0; c < kChunks; ++c) {
    const uint32_t i = c * kDedupNT + threadIdx.x;
    const bool mine = i < qall && part_of(ckey[c]) == part;
    bad |= i < qall && cop[c] > 2;
    bal[c] = __ballot(mine);
    if (lane == 0) wcnt[c][wid] = (uint32_t)__popcll(bal[c]);
  }
  __syncthreads();
  uint32_t base = 0;
#pragma unroll
  for (uint32_t c = 0; c < kChunks; ++c) {
    if (c >= nch) break;  // the same for the whole block
    uint32_t off = base, all = 0;
#pragma unroll
    for (uint32_t w = 0; w < kDedupNT / 64; ++w) {
      const uint32_t n = wcnt[c][w];
      off += w < wid ? n : 0;
      all += n;
    }
    if ((bal[c] >> lane) & 1) {
      const uint32_t at = off + (uint32_t)__popcll(bal[c] & ((1ull << lane) - 1));
      skey[at] = ckey[c];
      sidx[at] = ((c * kDedupNT + threadIdx.x) << 2) | (cop[c] & 3u);  // ordering by this is ordering by index
    }
    base += all;
  }
  __syncthreads();
  if (__any(bad) && lane == 0) a.ctl->reject = a.epoch;  // the same value from every writer
  const uint32_t q = base;  // commands in this partition
  if (q == 0) return;       // whole block
  if (q <= kDedupNT) {
    // One thread per command, in index order (position e).  The keys go to
    // the slots of an LDS hash table (a slot holds the position of one of
    // its key's commands), which gives each key its first command (the
    // leader of all of them) and its last PUT/DEL (the leader's last
    // write).  A command's previous write is the last PUT/DEL of its key
    // before it: within its wave from the ballot of the lanes sharing its
    // slot, else from the waves before it, swept in order.
    __shared__ uint32_t htab[kHashSlots];   // position + 1 of a command of the slot's key, 0 = empty
    __shared__ uint32_t hfirst[kHashSlots];  // first position of the slot's key
    __shared__ uint32_t hlast[kHashSlots];   // last PUT/DEL position + 1, 0 = none
    __shared__ uint32_t hrun[kHashSlots];    // the sweep: last PUT/DEL position + 1 in the waves so far
    for (uint32_t t = threadIdx.x; t < kHashSlots; t += kDedupNT) {
      htab[t] = 0;
      hfirst[t] = kNone;
      hlast[t] = 0;
      hrun[t] = 0;
    }
    __syncthreads();
    const uint32_t e = threadIdx.x;
    const bool real = e < q;
    const uint64_t key = real ? skey[e] : 0;
    const uint32_t pe = real ? sidx[e] : 0;
    const bool isw = real && (pe & 3u);
    uint32_t slot = kNone;
    if (real) {
      // at most q <= kDedupNT < kHashSlots keys: every probe sequence ends
      uint32_t h = (uint32_t)key_mix(key) & (kHashSlots - 1);
      for (uint32_t probe = 0; probe < kHashSlots; ++probe) {
        const uint32_t prev = atomicCAS(&htab[h], 0u, e + 1);
        if (prev == 0 || skey[prev - 1] == key) {
          slot = h;
          break;
        }
        h = (h + 1) & (kHashSlots - 1);
      }
      atomicMin(&hfirst[slot], e);
      if (isw) atomicMax(&hlast[slot], e + 1);
    }
    // lanes of this wave holding the same key, one round per distinct key
    uint64_t peers = 0;
    for (uint64_t todo = __ballot(real); todo;) {
      const uint32_t src = (uint32_t)__builtin_ctzll(todo);
      const uint32_t ss = (uint32_t)__builtin_amdgcn_readlane((int)slot, (int)src);
      const bool same = real && slot == ss;
      const uint64_t m = __ballot(same);
      if (same) peers = m;
      todo &= ~m;
    }
    const uint64_t kw = peers & __ballot(isw);  // this key's PUT/DELs in the wave
    const uint64_t below = kw & ((1ull << lane) - 1);
    uint32_t pwp = below ? (e - lane) + (63 - (uint32_t)__builtin_clzll(below)) + 1 : 0;  // position + 1
    const bool wave_last_w = isw && (kw >> lane) == 1;  // no later PUT/DEL of the key in the wave
    const uint32_t nw = (q + 63) / 64;
    for (uint32_t w = 0; w < nw; ++w) {
      if (wid == w && real) {
        if (!pwp) pwp = hrun[slot];
        if (wave_last_w) hrun[slot] = e + 1;  // after every lane's read: the wave's LDS ops are in order
      }
      __syncthreads();
    }
    if (real) {
      const uint32_t me = pe >> 2;
      const uint32_t f = hfirst[slot];
      leader[me] = sidx[f] >> 2;
      prevw[me] = pwp ? sidx[pwp - 1] >> 2 : kNone;
      if (f == e) lastw[me] = hlast[slot] ? sidx[hlast[slot] - 1] >> 2 : kNone;
    }
    return;
  }
  // Larger partitions (hot keys): sort the (key, index) pairs.
  uint32_t npad = 1;
  while (npad < q) npad <<= 1;
  uint64_t k[kDedupPer];
  uint32_t x[kDedupPer];
  const uint32_t r0 = threadIdx.x * kDedupPer;
#pragma unroll
  for (uint32_t e = 0; e < kDedupPer; ++e) {
    const uint32_t r = r0 + e;
    const bool real = r < q;
    k[e] = real ? skey[r] : kNone64;
    x[e] = real ? sidx[r] : kNone;  // command index << 2 | op
  }
  __syncthreads();  // the sort reuses skey / sidx
  dedup_sort(k, x, npad, skey, sidx);
  // Fold structure.  Each thread owns kDedupPer consecutive sorted
  // positions; positions are stored +1 so that 0 means "none".  The payload
  // is index << 2 | op.
  uint32_t rs[kDedupPer], wp[kDedupPer];
  uint32_t run = 0, wmax = 0;
  for (uint32_t t = 0; t < kDedupPer; ++t) {
    uint32_t r = r0 + t;
    if (r < q) {
      bool head = r == 0 || skey[r] != skey[r - 1];
      if (head) run = r + 1;
      rs[t] = run;
      wp[t] = wmax;  // writers strictly before r within this chunk
      if (sidx[r] & 3u) wmax = r + 1;
    } else {
      rs[t] = 0;
      wp[t] = 0;
    }
  }
  uint32_t run_in = block_excl<kDedupNT, true>(run, &tot);
  uint32_t w_in = block_excl<kDedupNT, true>(wmax, &tot);
  for (uint32_t t = 0; t < kDedupPer; ++t) {
    uint32_t r = r0 + t;
    if (r >= q) break;
    uint32_t start = rs[t] > run_in ? rs[t] : run_in;  // 1-based run start
    uint32_t w = wp[t] > w_in ? wp[t] : w_in;          // 1-based last writer before r
    const uint32_t me = sidx[r] >> 2;
    const uint32_t lead = sidx[start - 1] >> 2;
    leader[me] = lead;
    prevw[me] = (w != 0 && w >= start) ? (sidx[w - 1] >> 2) : kNone;
    bool tail = r + 1 == q || skey[r + 1] != skey[r];
    if (tail) {
      uint32_t wl = w;
      if (sidx[r] & 3u) wl = r + 1;
      lastw[lead] = (wl != 0 && wl >= start) ? (sidx[wl - 1] >> 2) : kNone;
    }
  }
}

// ---------------------------------------------------------------------------
// fetch: one wave per command
// ---------------------------------------------------------------------------



// Command i's fetch, by one whole wave (a sealed map decrypts its pages in
// the wave's LDS page pg).  EAGER (command i is a leader): each lane loads
// its rows' mask, keys and pairs at once, one round trip instead of three.
template <bool SEALED, bool EAGER = false>
__device__ __forceinline__ void fetch_cmd(const FetchArgs& a, uint32_t i, uint64_t* pg) {
  const uint32_t lane = threadIdx.x & 63;
  if (a.ctl->reject == a.epoch || a.ctl->err) return;
  const uint2 fp = a.fpair[i];  // F(s), from the dedup kernel
  const uint32_t f1 = fp.x, f2 = fp.y;
  const uint64_t key = a.keys[i];
  const bool is_leader = a.leader[i] == i;
  // key search (Sec. 5.1 step 3): d rows, 16 lanes per row, 2 slots per lane
  bool hit = false;
  uint32_t hrow = 0, hslot = 0, p1 = f1, p2 = f2;
  if (EAGER || is_leader) {
    const uint4 rw = a.rows[i];
    const uint32_t j = lane >> 4;
    const uint32_t row = j == 0 ? rw.x : j == 1 ? rw.y : j == 2 ? rw.z : rw.w;
    const uint32_t s0 = (lane & 15) * 2;
    bool m0 = false, m1 = false;
    uint2 pp0 = make_uint2(0, 0), pp1 = make_uint2(0, 0);
    if (j < a.d) {
      const uint32_t mk = a.pm_mask[row];
      if (EAGER) {
        const uint64_t* kr = a.pm_key + (uint64_t)row * a.W;
        const uint2* pr = a.pm_pair + (uint64_t)row * a.W;
        const uint64_t k0 = s0 < a.W ? kr[s0] : 0, k1 = s0 + 1 < a.W ? kr[s0 + 1] : 0;
        if (s0 < a.W) pp0 = pr[s0];
        if (s0 + 1 < a.W) pp1 = pr[s0 + 1];
        m0 = s0 < a.W && ((mk >> s0) & 1) && k0 == key;
        m1 = s0 + 1 < a.W && ((mk >> (s0 + 1)) & 1) && k1 == key;
      } else {
        if (s0 < a.W && ((mk >> s0) & 1)) m0 = a.pm_key[(uint64_t)row * a.W + s0] == key;
        if (s0 + 1 < a.W && ((mk >> (s0 + 1)) & 1)) m1 = a.pm_key[(uint64_t)row * a.W + s0 + 1] == key;
      }
    }
    const uint64_t bal = __ballot(m0 || m1);
    if (bal) {
      const uint32_t src = __builtin_ctzll(bal);
      const uint32_t slot = s0 + (m0 ? 0 : 1);
      hrow = __shfl(row, src, 64);
      hslot = __shfl(slot, src, 64);
      hit = true;
      if (EAGER) {
        const uint2 mp = m0 ? pp0 : pp1;
        p1 = __shfl(mp.x, src, 64);
        p2 = __shfl(mp.y, src, 64);
      } else {
        const uint2 pp = a.pm_pair[(uint64_t)hrow * a.W + hslot];
        p1 = pp.x;
        p2 = pp.y;
      }
    }
  }
  // value access (Sec. 5.1 step 4): both bins, whole.  Plain maps issue
  // both bins' first page words, stash lists and outbox marks at once
  // (nothing they read changes during the fetch, but pages the previous
  // batch rebuilt, which come from the outbox below).  A pinned host
  // store's pages are read at their turn instead: twice the reads in
  // flight crowd out the link's other direction, which carries the send.
  uint64_t pre0[2] = {0, 0}, pre1[2] = {0, 0}, pws[2] = {0, 0};
  uint32_t pcnt[2] = {0, 0}, pidx[2] = {kNone, kNone};
  if (!SEALED) {
#pragma unroll
    for (uint32_t r = 0; r < 2; ++r) {
      const uint32_t b = r ? p2 : p1;
      const bool host = b >= a.K;
      const bool pooled = a.decomp && !host;  // decomposed HBM bin: its list only
      const uint64_t* src = host ? a.obs + (uint64_t)(b - a.K) * a.pw : a.hbm + (uint64_t)b * a.pw;
      if (!pooled && (!host || a.pre_host)) {
        pre0[r] = lane < a.pw ? src[lane] : 0;
        pre1[r] = lane + 64 < a.pw ? src[lane + 64] : 0;
      }
      if (host || pooled) {
        pcnt[r] = a.rev_cnt[b];
        pidx[r] = lane < 2 * a.Z ? a.rev_idx[(uint64_t)b * 2 * a.Z + lane] : kNone;
      }
      if (host && a.ov_epoch) pws[r] = a.wslot[b - a.K];
    }
  }
  bool found = false;
#pragma unroll
  for (uint32_t role = 0; role < 2; ++role) {
    const uint32_t b = role ? p2 : p1;
    const uint32_t slot = 2 * i + role;
    const bool host = b >= a.K;
    if (lane == 0) {
      a.cand_bin[slot] = b;
      atomicMax((unsigned long long*)&a.claim[b], (unsigned long long)claim_tag(a.epoch, slot));
      if (a.tlog_r) a.tlog_r[slot] = host ? (uint32_t)(b - a.K) : kNone;
    }
    const uint64_t* src = host ? a.obs + (uint64_t)(b - a.K) * a.pw : a.hbm + (uint64_t)b * a.pw;
    uint64_t* stg = a.stage + (uint64_t)slot * a.pw;
    bool fresh = false;  // rebuilt by the previous batch, whose send may still run
    if (host && a.ov_epoch) {
      const uint64_t ws = SEALED ? a.wslot[b - a.K] : pws[role];
      if ((uint32_t)(ws >> 32) == a.ov_epoch) {
        // The store's copy is read all the same (the trace does not change),
        // but the page itself comes from the outbox.
        const volatile uint64_t* hv = src;
        uint64_t sink = 0;
        for (uint64_t w = lane; w < a.pw; w += 64) sink ^= hv[w];
        (void)sink;
        src = a.outbox + (uint64_t)(uint32_t)ws * a.pw;
        fresh = true;
      }
    }
    if (SEALED && a.tags && host && !fresh) {
      // Sealed page: copy it into this wave's LDS, check its tag under the
      // write count kept in HBM, and decrypt it there; the rest reads the
      // plain page from LDS.
      for (uint64_t w = lane; w < a.pw; w += 64) pg[w] = src[w];
      wave_sync();
      const uint32_t page = b - (uint32_t)a.K;
      const uint64_t ver = a.pver[page];
      uint32_t key[8], ks[16], otk[8], tag[4];
#pragma unroll
      for (int j = 0; j < 8; ++j) key[j] = a.ctl->skey[j];
      chacha_first_pass(key, page, (uint32_t)ver, (uint32_t)(ver >> 32), ks, otk);
      poly_page_tag(pg, (uint32_t)a.pw, otk, tag);
      const bool ok = a.tags[2 * (uint64_t)page] == ((uint64_t)tag[0] | ((uint64_t)tag[1] << 32)) &&
                      a.tags[2 * (uint64_t)page + 1] == ((uint64_t)tag[2] | ((uint64_t)tag[3] << 32));
      if (!ok && lane == 0) set_err(a.ctlw, kErrTamper);
      wave_sync();
      chacha_page_xor(pg, (uint32_t)a.pw, ks, key, page, (uint32_t)ver, (uint32_t)(ver >> 32));
      wave_sync();
      src = pg;
    }
    const bool pooled = a.decomp && !host;  // no page: it reads as empty
    const bool pre = !SEALED && !fresh && (!host || a.pre_host);  // the page words loaded above are the page's
    const uint64_t v0 = pooled ? 0 : (pre ? pre0[role] : (lane < a.pw ? src[lane] : 0));
    if (host && lane < a.pw) stg[lane] = v0;
    // find the key among the page's slots (lanes 1..Z hold the keys)
    const bool search = is_leader && hit && !found;
    int fslot = -1;
    if (search) {
      const uint64_t mask = __shfl(v0, 0, 64);
      const bool m = lane >= 1 && lane <= a.Z && ((mask >> (lane - 1)) & 1) && v0 == key;
      const uint64_t bal = __ballot(m);
      if (bal) fslot = (int)__builtin_ctzll(bal) - 1;
    }
    const uint64_t vlo = 1 + a.Z + (uint64_t)(fslot < 0 ? 0 : fslot) * a.vw;
    if (fslot >= 0 && lane >= vlo && lane < vlo + a.vw) a.fval[(uint64_t)i * a.vw + (lane - vlo)] = v0;
    for (uint64_t wi = lane + 64; !pooled && wi < a.pw; wi += 64) {
      const uint64_t v = (pre && wi < 128) ? pre1[role] : src[wi];
      if (host) stg[wi] = v;
      if (fslot >= 0 && wi >= vlo && wi < vlo + a.vw) a.fval[(uint64_t)i * a.vw + (wi - vlo)] = v;
    }
    if (fslot >= 0) {
      found = true;
      if (lane == 0) {
        atomicOr((unsigned long long*)&a.rmask[b], (unsigned long long)(1ull << fslot));
        atomicSub(&a.load[b], 1u);
        atomicSub(&a.load0[b], 1u);
      }
    } else if (search && (host || pooled)) {
      // the stash items listed for this bin (all of a decomposed HBM bin's items)
      const uint32_t cnt_raw = SEALED ? a.rev_cnt[b] : pcnt[role];
      const uint32_t cnt = cnt_raw < 2 * a.Z ? cnt_raw : 2 * a.Z;
      int fe = -1;
      for (uint32_t base = 0; base < cnt; base += 64) {
        const uint32_t l = base + lane;
        uint32_t e = kNone;
        bool m = false;
        if (l < cnt) {
          e = (!SEALED && base == 0) ? pidx[role] : a.rev_idx[(uint64_t)b * 2 * a.Z + l];
          m = !a.st_dead[e] && a.st_key[e] == key;
        }
        const uint64_t bal = __ballot(m);
        if (bal && fe < 0) fe = (int)__shfl(e, (int)__builtin_ctzll(bal), 64);
      }
      if (fe >= 0) {
        found = true;
        for (uint32_t o = lane; o < a.vw; o += 64) a.fval[(uint64_t)i * a.vw + o] = a.st_val[(uint64_t)fe * a.vw + o];
        if (lane == 0) {
          a.st_dead[fe] = 1;
          atomicSub(&a.load[b], 1u);
          atomicSub(&a.load0[b], 1u);
          if (pooled) atomicAdd(&a.ctlw->b_hbm_rm, 1u);
        }
      }
    }
  }
  if (lane == 0 && is_leader) {
    a.hit[i] = hit;
    a.hrow[i] = hrow;
    a.hslot[i] = hslot;
    a.found[i] = found;
    if (hit && !found) set_err(a.ctlw, kErrBroken);
    if (a.fast && hit) {
      const uint32_t lw = a.lastw[i];
      if (!(lw != kNone ? a.ops[lw] == 1 : found)) {  // deletes come before the inserts of this batch
        atomicAnd(&a.pm_mask_w[hrow], ~(1u << hslot));
        atomicAdd(&a.ctlw->b_del, 1u);
      }
    }
  }
}

template <bool MULTI, bool SEALED>
__global__ __launch_bounds__(256) void k_acc_fetch(FetchArgs a1, const AccessPlan* tab) {
  BOLT_PICK(FetchArgs, fa);
  extern __shared__ uint64_t fdyn[];
  uint64_t* const pg = fdyn + (uint64_t)(threadIdx.x >> 6) * a.pw;
  if (blockIdx.x < a.ship_blocks) {  // the previous batch's send (in a many-map launch, this map's)
    if (SEALED && a.ship.tags)
      ship_slots<true>(a.ship, blockIdx.x * 4 + (threadIdx.x >> 6), a.ship_blocks * 4, pg);
    else
      ship_slots<false>(a.ship, blockIdx.x * 4 + (threadIdx.x >> 6), a.ship_blocks * 4, nullptr);
    return;
  }
  const uint32_t i = (blockIdx.x - a.ship_blocks) * 4 + (threadIdx.x >> 6);
  if (i < a.q) fetch_cmd<SEALED>(a, i, pg);
}

// Claims a free slot of row r for (key, pair); false when the row is full.
__device__ __forceinline__ bool pm_claim(uint32_t* pm_mask, uint64_t* pm_key, uint2* pm_pair, uint32_t r, uint32_t W,
                                         uint64_t key, uint2 pair) {
  const uint32_t full = W >= 32 ? 0xFFFFFFFFu : ((1u << W) - 1);
  for (uint32_t tries = 0; tries < 32; ++tries) {
    const uint32_t mk = ld_acq32(&pm_mask[r]);
    const uint32_t free = ~mk & full;
    if (!free) return false;
    const uint32_t bit = free & (0u - free);
    const uint32_t prev = atomicOr(&pm_mask[r], bit);
    if (!(prev & bit)) {
      const uint32_t slot = __builtin_ctz(bit);
      pm_key[(uint64_t)r * W + slot] = key;
      pm_pair[(uint64_t)r * W + slot] = pair;
      return true;
    }
  }
  return false;
}

// ---------------------------------------------------------------------------
// resolve: responses and final states (one thread per command)
// ---------------------------------------------------------------------------



// What resolve hands a placement in the same thread: the command's final
// state as place reads it (0 unless it leads its key) and the key's bin.
struct Settled {
  uint32_t fin = 0, chosen = 0;
};

// Command i's response and, for a leader, its key's final state, by one
// thread (live: i < q); every lane of the wave calls it.  set, when given,
// also receives the state and bin (a placement in the same thread).
__device__ __forceinline__ void resolve_cmd(const ResolveArgs& a, uint32_t i, Settled* set = nullptr) {
  const bool live = i < a.q;
  if (a.ctl->reject == a.epoch || a.ctl->err) {
    if (live) {
      a.status[i] = 0xFF;
      for (uint32_t o = 0; o < a.vw; ++o) a.vals_out[(uint64_t)i * a.vw + o] = 0;
    }
    return;
  }
  if (live) {
    const uint32_t L = a.leader[i], w = a.prevw[i];
    const bool present = w != kNone ? a.ops[w] == 1 : a.found[L] != 0;
    const uint64_t* src = w != kNone ? a.vals_in + (uint64_t)w * a.vw : a.fval + (uint64_t)L * a.vw;
    const uint8_t op = a.ops[i];
    uint8_t st;
    if (op == 0) st = present ? 1 : 0;
    else if (op == 1) st = present ? 1 : 2;
    else st = present ? 3 : 0;
    a.status[i] = st;
    const bool give = op == 0 && present;
    uint64_t* out = a.vals_out + (uint64_t)i * a.vw;
    for (uint32_t o = 0; o < a.vw; ++o) out[o] = give ? src[o] : 0;
    if (L == i) {
      // final state of the key at the end of the batch
      const uint32_t lw = a.lastw[i];
      const bool fp = lw != kNone ? a.ops[lw] == 1 : a.found[i] != 0;
      const bool h = a.hit[i] != 0;
      const uint32_t fin = (fp ? 1u : 0u) | (h ? 2u : 0u);
      a.fin[i] = fin;
      if (set) set->fin = fin;
      if (a.fast && fp) {  // P2C over the post-removal loads (one round)
        const uint2 rp = a.rpair[i];
        const uint32_t b = a.load[rp.y] < a.load[rp.x] ? rp.y : rp.x;
        a.chosen[i] = b;
        if (set) set->chosen = b;
      }
    }
  }
}

template <bool MULTI>
__global__ __launch_bounds__(256) void k_acc_resolve(ResolveArgs a1, const AccessPlan* tab) {
  BOLT_PICK(ResolveArgs, rv);
  if (carry_ship<MULTI>(a.ship, a.ship_blocks)) return;
  resolve_cmd(a, (blockIdx.x - (MULTI ? 0 : a.ship_blocks)) * blockDim.x + threadIdx.x);
}

// ---------------------------------------------------------------------------
// place: stash entries, position-map updates, and in the one-round case the
// P2C loads and the row of every insert (one thread per command)
// ---------------------------------------------------------------------------



// Command i's placement, by one thread; every lane of the wave calls it.
// in: the state and bin from resolve_cmd in the same thread (else they are
// read from the batch's arrays).
__device__ __forceinline__ void place_cmd(const PlaceArgs& a, uint32_t i, const Settled* in = nullptr) {
  if (a.ctl->reject == a.epoch || a.ctl->err) return;  // the same for the whole wave
  bool placed = false, ins = false, to_hbm = false;
  uint32_t fin = 0, b = 0, lw = kNone, old = 0, ls = 0;
  uint64_t key = 0;
  if (i < a.q) {
    a.cand_bin[2 * a.q + i] = kNone;
    a.rowsel[i] = kNone;
    fin = in ? in->fin : (a.leader[i] == i ? a.fin[i] : 0);
    if (fin & 1) {
      // Every atomic and load that does not wait on another is issued
      // first; the capacity checks come last (a failure poisons the map,
      // whose state is then never read again).
      b = in ? in->chosen : a.chosen[i];
      lw = a.lastw[i];
      key = a.keys[i];
      old = a.several ? 0 : atomicAdd(&a.load[b], 1u);
      ls = atomicAdd(&a.rev_cnt[b], 1u);
      if (b < a.K && !a.decomp) {  // HBM bins are rebuilt in this batch
        a.cand_bin[2 * a.q + i] = b;
        atomicMax((unsigned long long*)&a.claim[b], (unsigned long long)claim_tag(a.epoch, 2 * a.q + i));
      }
      to_hbm = a.decomp && b < a.K;  // a decomposed HBM bin keeps the entry listed
      if (fin & 2) {
        a.pm_pair[(uint64_t)a.hrow[i] * a.W + a.hslot[i]] = a.rpair[i];
      } else if (!a.several) {
        // insert: the least loaded of d rows after this batch's deletes
        const uint4 rw = a.rows[i];
        uint32_t best = rw.x;
        uint32_t bc = __popc(a.pm_mask[best]);
        for (uint32_t j = 1; j < a.d; ++j) {
          const uint32_t r = j == 1 ? rw.y : j == 2 ? rw.z : rw.w;
          const uint32_t c = __popc(a.pm_mask[r]);
          if (c < bc) {
            bc = c;
            best = r;
          }
        }
        a.rowsel[i] = best;
        ins = true;
      }
    }
  }
  // the item goes to a fresh stash entry listed under bin b (the wave takes
  // its lanes' pool entries together, from a window where its index leads)
  const uint32_t e_pool =
      a.decomp ? kNone : pool_alloc_wave(a.st_used, a.PW, alloc_hash(a.epoch, i - (threadIdx.x & 63)), (fin & 1) != 0);
  if (fin & 1) {
    const uint32_t e = a.decomp ? ring_alloc(a.ctl, a.ring, a.P) : e_pool;
    const uint64_t* src = lw != kNone ? a.vals_in + (uint64_t)lw * a.vw : a.fval + (uint64_t)i * a.vw;
    if (e != kNone) {
      a.st_key[e] = key;
      for (uint32_t x = 0; x < a.vw; ++x) a.st_val[(uint64_t)e * a.vw + x] = src[x];
      a.st_dest[e] = b;
      a.st_dead[e] = 0;
      if (ls < 2 * a.Z) a.rev_idx[(uint64_t)b * 2 * a.Z + ls] = e;
    }
    if ((!a.several && old + 1 > a.Z) || e == kNone || ls >= 2 * a.Z) set_err(a.ctl, kErrOverflow);
    placed = true;
  }
  if (!a.several) {  // k_acc_remap counts the several-round path's
    wave_count(&a.ctl->b_place, placed);
    wave_count(&a.ctl->b_ins, ins);
  }
  if (a.decomp) wave_count(&a.ctl->b_hbm_in, to_hbm);
}

template <bool MULTI>
__global__ __launch_bounds__(256) void k_acc_place(PlaceArgs a1, const AccessPlan* tab) {
  BOLT_PICK(PlaceArgs, pa);
  if (carry_ship<MULTI>(a.ship, a.ship_blocks)) return;
  place_cmd(a, (blockIdx.x - (MULTI ? 0 : a.ship_blocks)) * blockDim.x + threadIdx.x);
}

// Resolve and place in one launch (a one-map, one-round batch): each
// thread's placement needs only its own command's final state and bin,
// the choices read the loads as placement began (a copy the adds do not
// touch), and the deletes were made by the fetch.
__global__ __launch_bounds__(64) void k_acc_settle(ResolveArgs rv, PlaceArgs pa) {
  if (carry_ship<false>(pa.ship, pa.ship_blocks)) return;
  const uint32_t i = (blockIdx.x - pa.ship_blocks) * blockDim.x + threadIdx.x;
  Settled st;
  resolve_cmd(rv, i, &st);
  place_cmd(pa, i, &st);
}

// ---------------------------------------------------------------------------
// remap, several rounds (one workgroup): the steps that go in rounds, in
// round order.  Phase 0: P2C in rounds of ceil(B/16) (each placed key's bin
// to `chosen`, its load added) and the deletes, before k_acc_place; phase
// 1: the inserts in rounds of ceil(R/16), after it.
// ---------------------------------------------------------------------------

constexpr uint32_t kRemapNT = 1024;
constexpr uint32_t kRemapPer = kMaxBatch / kRemapNT;
// Maps of at most this many bins keep their loads in dynamic LDS through
// the P2C rounds of a several-round batch (a round holds ceil(B/16) keys, so
// small maps run many rounds: up to 1024 for a batch of 8192 on 128 bins),
// and one wave runs the rounds, at most kWaveKeys keys per lane.  With the
// round list beside it the workgroup holds 128 KiB of LDS.
constexpr uint32_t kRemapLdsBins = 24576;
constexpr uint32_t kWaveKeys = (kRemapLdsBins / 16 + 63) / 64;  // 24



template <bool MULTI>
__global__ __launch_bounds__(kRemapNT) void k_acc_remap(RemapArgs a1, const AccessPlan* tab, uint32_t phase,
                                                         uint32_t lds_bins) {
  BOLT_PICK(RemapArgs, ra);
  if (!a.enabled) return;
  __shared__ uint32_t tot;
  __shared__ uint32_t s_skip;
  if (threadIdx.x == 0) s_skip = (a.ctl->reject == a.epoch || a.ctl->err) ? 1 : 0;
  __syncthreads();
  if (s_skip) return;
  const uint32_t i0 = threadIdx.x * kRemapPer;
  uint32_t fin[kRemapPer];  // bit0 present at the end, bit1 mapped at the start
  uint32_t nplace_mine = 0, nins_mine = 0, ndel_mine = 0;
  for (uint32_t t = 0; t < kRemapPer; ++t) {
    const uint32_t i = i0 + t;
    fin[t] = (i < a.q && a.leader[i] == i) ? a.fin[i] : 0;
    nplace_mine += fin[t] & 1;
    nins_mine += (fin[t] & 3) == 1;
    ndel_mine += (fin[t] & 3) == 2;
  }
  const uint32_t place0 = block_excl<kRemapNT, false>(nplace_mine, &tot);
  const uint32_t nplace = tot;
  __syncthreads();
  const uint32_t ins0 = block_excl<kRemapNT, false>(nins_mine, &tot);
  const uint32_t nins = tot;
  __syncthreads();
  block_excl<kRemapNT, false>(ndel_mine, &tot);
  const uint32_t ndel = tot;
  __syncthreads();
  if (phase == 0) {
    // P2C in rounds of ceil(B/16) over the post-removal loads (Sec. 5.1 step 5).
    const uint64_t rs = (a.B + 15) / 16;
    uint32_t chosen[kRemapPer];
    // A map of at most lds_bins bins (the launch's dynamic LDS) keeps its
    // loads in LDS meanwhile (the only writer of this map's loads in this
    // launch is this workgroup), and one wave runs the rounds with no
    // workgroup barrier: the keys' pairs (packed, bins < 2^16) go to an LDS
    // list in placement order; per round the wave reads the list entries
    // and the loads of all its keys (at most kWaveKeys per lane), then adds
    // (a wave's LDS operations complete in order, so every read of a round
    // sees the loads at its start); each key's chosen bin goes back into its
    // list entry for the thread that holds the command.
    extern __shared__ uint32_t s_load[];
    __shared__ uint32_t s_list[kMaxBatch + 1];  // the last entry takes idle lanes' writes
    const bool lds_loads = a.B <= lds_bins && nplace > rs;  // the same for the whole workgroup
    if (lds_loads) {
      for (uint32_t b = threadIdx.x; b < a.B; b += kRemapNT) s_load[b] = ld_acq32(&a.load[b]);
      uint32_t o = place0;
      for (uint32_t t = 0; t < kRemapPer; ++t) {
        if (!(fin[t] & 1)) continue;
        const uint2 rp = a.rpair[i0 + t];
        s_list[o++] = rp.x | (rp.y << 16);
      }
      __syncthreads();
      const uint32_t K = (uint32_t)((rs + 63) / 64);  // keys a lane per round, the same for the workgroup
      if (threadIdx.x < 64 && K == 1) {
        // One key a lane: a round waits on one LDS round trip, its loads;
        // its list entries were read during the round before.  Lanes without
        // a key read valid bins (list entries only hold bins), add zero and
        // write to the spare last list entry.  Adds return nothing: a bin
        // past Z during the rounds is past it after them, as loads only grow
        // here, and is found then.
        const uint32_t lane = threadIdx.x;
        const bool in_round = lane < rs;
        uint32_t pk = in_round && lane < nplace ? s_list[lane] : 0;
        __builtin_amdgcn_s_waitcnt(0);  // nothing in flight when the loop starts
        for (uint32_t r0 = 0; r0 < nplace; r0 += (uint32_t)rs) {
          const uint32_t k = r0 + lane, kn = k + (uint32_t)rs;
          const bool mine = in_round && k < nplace;
          const uint32_t p1 = pk & 0xFFFFu, p2 = pk >> 16;
          // the next round's entries first: in order, they are back by the
          // time this round's loads are
          const uint32_t pk_next = s_list[kn < nplace ? kn : 0];
          __builtin_amdgcn_sched_barrier(0);
          const uint32_t l1 = s_load[p1], l2 = s_load[p2];
          const uint32_t ch = l2 < l1 ? p2 : p1;
          __builtin_amdgcn_wave_barrier();
          atomicAdd(&s_load[ch], mine ? 1u : 0u);
          s_list[mine ? k : kMaxBatch] = ch;
          __builtin_amdgcn_wave_barrier();
          pk = in_round ? pk_next : 0;
        }
      } else if (threadIdx.x < 64) {
        // Several keys a lane (the same rules)
        const uint32_t lane = threadIdx.x;
        for (uint32_t r0 = 0; r0 < nplace; r0 += (uint32_t)rs) {
          uint32_t ch[kWaveKeys];
          bool mine[kWaveKeys];
#pragma unroll
          for (uint32_t j = 0; j < kWaveKeys; ++j) {
            if (j >= K) break;
            const uint32_t off = j * 64 + lane, k = r0 + off;
            mine[j] = off < rs && k < nplace;
            const uint32_t pk = s_list[mine[j] ? k : kMaxBatch];
            const uint32_t p1 = mine[j] ? pk & 0xFFFFu : 0, p2 = mine[j] ? pk >> 16 : 0;
            const uint32_t l1 = s_load[p1], l2 = s_load[p2];
            ch[j] = l2 < l1 ? p2 : p1;
          }
          // every read of the round before any add
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_sched_barrier(0);
          asm volatile("" ::: "memory");
#pragma unroll
          for (uint32_t j = 0; j < kWaveKeys; ++j) {
            if (j >= K) break;
            atomicAdd(&s_load[ch[j]], mine[j] ? 1u : 0u);
            s_list[mine[j] ? r0 + j * 64 + lane : kMaxBatch] = ch[j];
          }
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_sched_barrier(0);
          asm volatile("" ::: "memory");
        }
      }
      __syncthreads();
      o = place0;
      for (uint32_t t = 0; t < kRemapPer; ++t)
        if (fin[t] & 1) chosen[t] = s_list[o++];
      // the loads go back, and a bin past Z is found on the way
      bool over = false;
      for (uint32_t b = threadIdx.x; b < a.B; b += kRemapNT) {
        const uint32_t l = s_load[b];
        over |= l > a.Z;
        a.load[b] = l;
      }
      if (over) set_err(a.ctl, kErrOverflow);
    } else {
      // The loads in global memory: the workgroup runs the rounds, its
      // threads' keys of a round read, a barrier, then the adds.
      for (uint64_t r0 = 0; r0 < nplace; r0 += rs) {
        uint32_t o = place0;
        for (uint32_t t = 0; t < kRemapPer; ++t) {
          if (!(fin[t] & 1)) continue;
          if (o >= r0 && o < r0 + rs) {
            const uint2 rp = a.rpair[i0 + t];
            const uint32_t l1 = ld_acq32(&a.load[rp.x]);
            const uint32_t l2 = ld_acq32(&a.load[rp.y]);
            chosen[t] = l2 < l1 ? rp.y : rp.x;
          }
          ++o;
        }
        __syncthreads();
        o = place0;
        bool over = false;  // one error report after the adds, so that they issue together
        for (uint32_t t = 0; t < kRemapPer; ++t) {
          if (!(fin[t] & 1)) continue;
          if (o >= r0 && o < r0 + rs) over |= atomicAdd(&a.load[chosen[t]], 1u) + 1 > a.Z;
          ++o;
        }
        if (over) set_err(a.ctl, kErrOverflow);
        __threadfence();
        __syncthreads();
      }
    }
    // each placed key's bin for k_acc_place (which lists the item under it),
    // and the deletes, which the inserts of phase 1 see
    for (uint32_t t = 0; t < kRemapPer; ++t) {
      const uint32_t i = i0 + t;
      if (fin[t] & 1) a.chosen[i] = chosen[t];
      if ((fin[t] & 3) == 2) atomicAnd(&a.pm_mask[a.hrow[i]], ~(1u << a.hslot[i]));
    }
    if (threadIdx.x == 0) {
      a.ctl->b_place = nplace;
      a.ctl->b_ins = nins;
      a.ctl->b_del = ndel;
    }
    return;
  }
  // Phase 1: the inserts, in rounds of ceil(R/16) that see the row loads at
  // their start; the least loaded of d rows, ties to the lowest choice
  const uint64_t rsm = (a.R + 15) / 16;
  uint32_t rowsel[kRemapPer];
  for (uint64_t r0 = 0; r0 < nins; r0 += rsm) {
    uint32_t io = ins0;
    for (uint32_t t = 0; t < kRemapPer; ++t) {
      if ((fin[t] & 3) != 1) continue;
      if (io >= r0 && io < r0 + rsm) {
        const uint4 rw = a.rows[i0 + t];
        uint32_t best = rw.x;
        uint32_t bc = __popc(ld_acq32(&a.pm_mask[best]));
        for (uint32_t j = 1; j < a.d; ++j) {
          const uint32_t r = j == 1 ? rw.y : j == 2 ? rw.z : rw.w;
          const uint32_t c = __popc(ld_acq32(&a.pm_mask[r]));
          if (c < bc) {
            bc = c;
            best = r;
          }
        }
        rowsel[t] = best;
      }
      ++io;
    }
    __syncthreads();
    io = ins0;
    for (uint32_t t = 0; t < kRemapPer; ++t) {
      if ((fin[t] & 3) != 1) continue;
      if (io >= r0 && io < r0 + rsm) {
        if (!pm_claim(a.pm_mask, a.pm_key, a.pm_pair, rowsel[t], a.W, a.keys[i0 + t], a.rpair[i0 + t]))
          set_err(a.ctl, kErrOverflow);
      }
      ++io;
    }
    __threadfence();
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// write-back with eviction: one wave per candidate slot
// ---------------------------------------------------------------------------



constexpr uint32_t kWbItems = 192;  // Z survivors + 2Z listed stash entries, Z <= 62
constexpr uint32_t kFreeBuckets = 256;

// Dynamic LDS of one write-back wave: the old page, then the item lists.
__host__ __device__ constexpr uint64_t wb_lds_bytes(uint64_t pw) { return pw * 8 + kWbItems * 12 + 64 * 4; }

// One wave (one workgroup) per candidate slot.  The elected writer copies
// the bin's old page into LDS (observable pages from the stage the fetch
// wrote, HBM bins from HBM), so the rebuilt page can be written in place
// without any device-wide fence.  HBM bins are rebuilt in place; an
// observable page is rebuilt into the outbox at the writer's slot, for
// k_acc_ship to send.
// Candidate slot s's rebuild, by one whole wave with its own dynamic LDS
// (wb_lds_bytes, plus a page for a sealed map) at dyn.  MAY_SEAL = false
// leaves out the sealing of directly written pages (plain maps only).
template <bool MAY_SEAL>
__device__ __forceinline__ void compose_slot(const WbArgs& a, uint32_t s, uint64_t* dyn) {
  uint64_t* old = dyn;
  uint64_t* ikey = dyn + a.pw;
  uint32_t* isrc = reinterpret_cast<uint32_t*>(ikey + kWbItems);
  uint32_t* by_rank = isrc + kWbItems;
  const uint32_t lane = threadIdx.x & 63;
  if (lane == 0 && s < 2 * a.q) a.ship_page[s] = kNone;
  if (lane == 0 && s < 3 * a.q && a.decomp) a.rfree_n[s] = 0;  // this slot returns nothing unless it rebuilds
  if (s >= 3 * a.q || a.ctl->reject == a.epoch || a.ctl->err) return;  // whole wave
  // The placement's adds are done: carry them into the copy.  Only a batch
  // that went through (no reject, no error) has its final states and bins.
  if (lane == 0 && s >= 2 * a.q) {
    const uint32_t i = s - 2 * a.q;
    if (a.leader[i] == i && (a.fin[i] & 1)) {
      const uint32_t b = a.chosen[i];
      a.load0[b] = a.load[b];
    }
  }
  const uint32_t b = a.cand_bin[s];
  if (b == kNone) return;  // whole wave
  const bool host = b >= a.K;
  if (host && s >= 2 * a.q) {  // observable bins are only claimed by fetch slots
    if (lane == 0) set_err(a.ctl, kErrBroken);
    return;
  }
  // The election's outcome and the bin's data are loaded together (a slot
  // that lost the election drops what it read).
  const uint64_t cl = a.claim[b];
  const bool pooled = a.decomp && !host;  // a decomposed HBM bin: its list only
  const uint64_t* src = host ? a.stage + (uint64_t)s * a.pw : a.hbm + (uint64_t)b * a.pw;
  for (uint64_t w = lane; w < a.pw; w += 64) old[w] = pooled ? 0 : src[w];
  const uint64_t rm = a.rmask[b];
  const uint32_t cnt_raw = a.rev_cnt[b];
  const uint32_t e_spec = lane < 2 * a.Z ? a.rev_idx[(uint64_t)b * 2 * a.Z + lane] : kNone;  // the bin's list row
  if (cl != claim_tag(a.epoch, s)) return;  // whole wave
  const uint32_t cnt = cnt_raw < 2 * a.Z ? cnt_raw : 2 * a.Z;
  wave_sync();
  const uint64_t keep = old[0] & ~rm;
  // survivors, in slot order
  if (lane < a.Z && ((keep >> lane) & 1)) {
    const uint32_t pos = __popcll(keep & ((1ull << lane) - 1));
    ikey[pos] = old[1 + lane];
    isrc[pos] = lane;  // page slot
  }
  const uint32_t n_surv = __popcll(keep);
  // every entry listed under the bin: live ones move in, all are freed
  uint32_t n_alive = 0;
  for (uint32_t base = 0; base < cnt; base += 64) {
    const uint32_t l = base + lane;
    uint32_t e = kNone;
    bool alive = false;
    if (l < cnt) {
      e = base == 0 ? e_spec : a.rev_idx[(uint64_t)b * 2 * a.Z + l];
      alive = !a.st_dead[e];
    }
    const uint64_t bal = __ballot(alive);
    if (alive) {
      const uint32_t pos = n_surv + n_alive + __popcll(bal & ((1ull << lane) - 1));
      if (pos < kWbItems) {
        ikey[pos] = a.st_key[e];
        isrc[pos] = 0x80000000u | e;
      }
    }
    n_alive += __popcll(bal);
  }
  const uint32_t n_items = n_surv + n_alive;
  if (n_items > a.Z) {  // the load bound was broken: report, write nothing
    if (lane == 0) set_err(a.ctl, kErrOverflow);
    return;
  }
  wave_sync();
  if (pooled) {
    // A decomposed HBM bin keeps its live entries listed (the first n_alive
    // list positions, all below 64, were read into e_spec before) and
    // returns the dead ones to the ring.
    uint32_t ndead = 0;
    for (uint32_t base = 0; base < cnt; base += 64) {
      const uint32_t l = base + lane;
      bool dead = false;
      uint32_t e = kNone;
      if (l < cnt) {
        e = base == 0 ? e_spec : a.rev_idx[(uint64_t)b * 2 * a.Z + l];
        dead = a.st_dead[e] != 0;
        if (dead) a.st_dead[e] = 0;
      }
      const uint64_t bal = __ballot(dead);
      if (dead) a.rfree[(uint64_t)s * 2 * a.Z + ndead + __popcll(bal & ((1ull << lane) - 1))] = e;
      ndead += __popcll(bal);
    }
    if (lane < n_alive) a.rev_idx[(uint64_t)b * 2 * a.Z + lane] = isrc[lane] & 0x7FFFFFFFu;
    if (lane == 0) {
      a.rmask[b] = 0;
      a.rev_cnt[b] = n_alive;
      a.rfree_n[s] = (uint8_t)ndead;
      if (ndead) atomicAdd(&a.freed[s % kFreeBuckets], ndead);
    }
    return;
  }
  // canonical order: ascending key
  if (lane < n_items) {
    const uint64_t mine = ikey[lane];
    uint32_t rank = 0;
    for (uint32_t j = 0; j < n_items; ++j) rank += ikey[j] < mine || (ikey[j] == mine && j < lane);
    by_rank[rank] = lane;
  }
  wave_sync();
  // HBM bin: in place.  Observable page: to the outbox, or straight to the
  // store when direct (a sealed one through LDS after the item lists).
  const bool seal = MAY_SEAL && host && a.direct && a.tags;
  uint64_t* const dst = host ? (a.direct ? a.obs + (uint64_t)(b - a.K) * a.pw : a.outbox + (uint64_t)s * a.pw)
                             : a.hbm + (uint64_t)b * a.pw;
  uint64_t* out = seal ? reinterpret_cast<uint64_t*>(reinterpret_cast<char*>(dyn) + wb_lds_bytes(a.pw)) : dst;
  for (uint64_t w = lane; w < a.pw; w += 64) {
    uint64_t v = 0;
    if (w == 0) {
      v = n_items >= 64 ? kNone64 : ((1ull << n_items) - 1);
    } else if (w <= a.Z) {
      const uint32_t j = (uint32_t)w - 1;
      v = j < n_items ? ikey[by_rank[j]] : 0;
    } else if (w < 1 + a.Z + (uint64_t)a.Z * a.vw) {
      const uint64_t off = w - 1 - a.Z;
      const uint32_t j = (uint32_t)(off / a.vw), o = (uint32_t)(off % a.vw);
      if (j < n_items) {
        const uint32_t from = isrc[by_rank[j]];
        v = (from & 0x80000000u) ? a.st_val[(uint64_t)(from & 0x7FFFFFFFu) * a.vw + o]
                                 : old[1 + a.Z + (uint64_t)from * a.vw + o];
      }
    }
    out[w] = v;
  }
  if (seal) {
    const uint32_t page = b - (uint32_t)a.K;
    const uint64_t ver = a.pver[page] + 1;
    uint32_t key[8], tag[4];
#pragma unroll
    for (int j = 0; j < 8; ++j) key[j] = a.ctl->skey[j];
    seal_page(out, (uint32_t)a.pw, key, page, ver, dst, tag);
    if (lane == 0) {
      a.tags[2 * (uint64_t)page] = (uint64_t)tag[0] | ((uint64_t)tag[1] << 32);
      a.tags[2 * (uint64_t)page + 1] = (uint64_t)tag[2] | ((uint64_t)tag[3] << 32);
      a.pver[page] = ver;
    }
  }
  // free every listed entry (its value was read above)
  for (uint32_t l = lane; l < cnt; l += 64) {
    const uint32_t e = l < 64 ? e_spec : a.rev_idx[(uint64_t)b * 2 * a.Z + l];
    a.st_dead[e] = 0;
    if (a.decomp)
      a.rfree[(uint64_t)s * 2 * a.Z + l] = e;  // staged; the finish returns it to the ring
    else
      pool_free(a.st_used, e);
  }
  if (lane == 0) {
    if (a.decomp) a.rfree_n[s] = (uint8_t)cnt;
    a.rmask[b] = 0;
    a.rev_cnt[b] = 0;
    if (cnt) atomicAdd(&a.freed[s % kFreeBuckets], cnt);
    if (host) {
      const uint32_t page = b - (uint32_t)a.K;
      if (!a.direct) {
        a.ship_page[s] = page;
        a.wslot[page] = ((uint64_t)a.epoch << 32) | s;
      }
      if (a.tlog_w) a.tlog_w[s] = page;
    }
  }
}

// One wave (one workgroup) per candidate slot; wave n of the launch takes
// slot s(n).  The remap slots [2q, 3q) come first (n < q): most have no bin
// and end at once, which frees wave slots early for the fetch slots [0, 2q)
// (n in [q, 3q)).  Launched last, they waited for the first round of fetch
// slots to end: a batch's 3q waves exceed what the device holds at once.
// The first ship_blocks workgroups send a slice of the previous batch's
// pages (from the other half of the outbox).  SEALED: some map of the
// launch seals its store.
template <bool MULTI, bool SEALED>
__global__ __launch_bounds__(64) void k_acc_compose(WbArgs a1, const AccessPlan* tab) {
  BOLT_PICK(WbArgs, wa);
  extern __shared__ uint64_t dyn[];
  if (carry_ship<MULTI>(a.ship, a.ship_blocks)) return;
  const uint32_t n = blockIdx.x - (MULTI ? 0 : a.ship_blocks);
  const uint32_t s = n < a.q ? 2 * a.q + n : (n < 3 * a.q ? n - a.q : n);
  compose_slot<SEALED>(a, s, dyn);
}

// ---------------------------------------------------------------------------
// finish: position-map inserts of the one-round case, then the counters
// ---------------------------------------------------------------------------



// Command i's position-map insert (one-round case).
__device__ __forceinline__ void finish_cmd(const FinishArgs& a, uint32_t i) {
  if (i < a.q && a.rowsel && a.rowsel[i] != kNone) {
    if (!pm_claim(a.pm_mask, a.pm_key, a.pm_pair, a.rowsel[i], a.W, a.keys[i], a.rpair[i]))
      set_err(a.ctl, kErrOverflow);
  }
}

// The batch's counter update, by one thread, given the stash entries the
// rebuild freed (ok: no error was set before the inserts).
__device__ __forceinline__ void finish_apply(const FinishArgs& a, bool ok, uint64_t freed) {
  Ctl* c = a.ctl;
  if (ok) {
    c->steps += a.q;
    // pool entries in use: the stash proper plus, in a decomposed store,
    // the HBM bins' items (hbm_live stays 0 otherwise)
    const uint64_t pool = c->pool_live + c->b_place - freed;
    c->pool_live = pool;
    const uint64_t hbm = c->hbm_live + c->b_hbm_in - c->b_hbm_rm;
    c->hbm_live = hbm;
    const uint64_t st = pool - hbm;
    c->stash_live = st;
    if (st > c->stash_hw) c->stash_hw = st;
    if (st > a.stash_bound || hbm > a.hbm_bound) c->err |= kErrOverflow;
    const uint64_t live = c->live + c->b_ins - c->b_del;
    c->live = live;
    if (live > a.cap) c->err |= kErrFull;
  }
  c->b_place = 0;
  c->b_ins = 0;
  c->b_del = 0;
  c->ring_head += c->ring_take;  // the ring: this batch's takes and returns
  c->ring_tail += c->ring_give;
  c->ring_take = 0;
  c->ring_give = 0;
  c->b_hbm_in = 0;
  c->b_hbm_rm = 0;
}

// The batch's counters, by one whole workgroup: the freed buckets summed
// and cleared; part is kFreeBuckets words of LDS.  Every batch leaves the
// buckets at zero.
__device__ __forceinline__ void finish_counters(const FinishArgs& a, bool ok, uint32_t* part) {
  for (uint32_t t = threadIdx.x; t < kFreeBuckets; t += blockDim.x) {
    part[t] = a.freed[t];
    a.freed[t] = 0;  // ready for the next batch
  }
  __syncthreads();
  for (uint32_t h = kFreeBuckets / 2; h > 0; h >>= 1) {
    for (uint32_t t = threadIdx.x; t < h; t += blockDim.x) part[t] += part[t + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) finish_apply(a, ok, part[0]);
}

// Decomposed store: workgroup bid of nb returns its share of the entries
// the rebuild slots staged to the ring's tail.  The 3q slots are split into
// nb contiguous ranges of at most kRetChunk slots (3q <= 768 nb for every
// launch: nb >= q / 256); entries go to the ring in slot order, so a range
// starts after every entry of the slots before it (summed here, each
// workgroup on its own).  The range's slot offsets go to LDS and each
// thread then copies every 256th entry, so no thread waits on a chain of
// loads.  The workgroup adds its count to ring_give.
constexpr uint32_t kRetChunk = 768;

__device__ __forceinline__ void ring_return(const FinishArgs& a, uint32_t bid, uint32_t nb) {
  const uint32_t n3 = 3 * a.q, per_wg = (n3 + nb - 1) / nb;
  const uint32_t lo = bid * per_wg < n3 ? bid * per_wg : n3, hi = lo + per_wg < n3 ? lo + per_wg : n3;
  __shared__ uint32_t pre[kRetChunk + 1];
  __shared__ uint32_t tot;
  if (hi - lo > kRetChunk) {  // not reached by the launches above
    if (threadIdx.x == 0) set_err(a.ctl, kErrOverflow);
    return;
  }
  // entries of the slots before the range: the counts are bytes, summed
  // sixteen per load, four loads in flight per thread
  const uint4* c16 = reinterpret_cast<const uint4*>(a.rfree_n);
  auto bytes4 = [](uint32_t x) {
    const uint32_t v = (x & 0x00FF00FFu) + ((x >> 8) & 0x00FF00FFu);
    return (v & 0xFFFFu) + (v >> 16);
  };
  auto bytes16 = [&](const uint4 v) { return bytes4(v.x) + bytes4(v.y) + bytes4(v.z) + bytes4(v.w); };
  const uint32_t full = lo >> 4;
  uint32_t acc[4] = {0, 0, 0, 0};
  uint32_t ci = threadIdx.x;
  for (; ci + 3 * 256 < full; ci += 4 * 256) {
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] += bytes16(c16[ci + k * 256]);
  }
  for (; ci < full; ci += 256) acc[0] += bytes16(c16[ci]);
  for (uint32_t s = (full << 4) + threadIdx.x; s < lo; s += 256) acc[1] += a.rfree_n[s];
  const uint32_t before = acc[0] + acc[1] + acc[2] + acc[3];
  block_excl<256, false>(before, &tot);
  const uint64_t at = a.ctl->ring_tail + tot;  // the tail moves only when the last workgroup is done
  // the range's counts, three consecutive slots per thread, and their offsets
  const uint32_t len = hi - lo, s0 = threadIdx.x * 3;
  uint32_t c[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) c[k] = s0 + k < len ? a.rfree_n[lo + s0 + k] : 0;
  uint32_t off = block_excl<256, false>(c[0] + c[1] + c[2], &tot);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (s0 + k < len) pre[s0 + k] = off;
    off += c[k];
  }
  const uint32_t total = tot;
  if (threadIdx.x == 0) pre[len] = total;
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < total; i += 256) {
    // the slot x with pre[x] <= i < pre[x + 1]: the last offset <= i
    uint32_t x = 0, span = len;
    while (span > 0) {
      const uint32_t h = span >> 1;
      if (pre[x + h + 1] <= i) {
        x += h + 1;
        span -= h + 1;
      } else {
        span = h;
      }
    }
    a.ring[(at + i) % a.P] = a.rfree[(uint64_t)(lo + x) * a.Z2 + (i - pre[x])];
  }
  if (threadIdx.x == 0 && total) atomicAdd(&a.ctl->ring_give, total);
}

template <bool MULTI>
__global__ __launch_bounds__(256) void k_acc_finish(FinishArgs a1, const AccessPlan* tab) {
  BOLT_PICK(FinishArgs, fn);
  if (carry_ship<MULTI>(a.ship, a.ship_blocks)) return;
  const uint32_t bid = blockIdx.x - (MULTI ? 0 : a.ship_blocks);
  if (a.ctl->reject == a.epoch) return;
  const bool ok = !a.ctl->err;
  if (ok) finish_cmd(a, bid * blockDim.x + threadIdx.x);
  __shared__ uint32_t part[kFreeBuckets];
  if (!a.decomp) {  // (the plan's flag: the same for the whole workgroup)
    if (bid == 0) finish_counters(a, ok, part);
    return;
  }
  // Every workgroup returns its share of the staged entries; the last one
  // done (a counter, no waiting) applies the batch's counters, when every
  // share is in the ring and ring_give is whole.
  const uint32_t nb = gridDim.x - (MULTI ? 0 : a.ship_blocks);
  ring_return(a, bid, nb);
  __threadfence();
  __syncthreads();
  __shared__ uint32_t last;
  if (threadIdx.x == 0) last = atomicAdd(&a.ctl->fin_done, 1u) == nb - 1;
  __syncthreads();
  if (!last) return;
  __threadfence();
  if (threadIdx.x == 0) a.ctl->fin_done = 0;
  finish_counters(a, ok, part);
}

// ---------------------------------------------------------------------------
// a batch of one command on a plain map, in one workgroup
// ---------------------------------------------------------------------------

// Three waves run the batched kernels' steps in their order; each step ends
// at a workgroup barrier, which makes what the step stored or changed by
// atomics in global memory visible to the whole workgroup (all its waves
// share one CU and its L1).  The dedup of one command is trivial; its two
// PRFs run on waves 1 and 2; fetch, resolve and place on wave 0 (waves 1
// and 2 warm L2 for the later steps meanwhile); the rebuild of candidate
// slot s on wave s; then the insert and the counters.  A wave's dynamic LDS
// for the rebuild is wb_stride bytes.
constexpr uint32_t kSoloNT = 192;

__device__ __forceinline__ void solo_step() { __syncthreads(); }

// Waves 1 and 2 while wave 0 fetches: loads of lines that the later steps
// read or change by atomics, so that they find them in L2 rather than HBM.
// The values are folded into one word, stored only if it equals a constant
// (which changes nothing even then).
__device__ __forceinline__ void solo_warm(const FetchArgs& fa, const PlaceArgs& pa, uint32_t wave, uint32_t lane) {
  uint64_t acc = 0;
  if (wave == 1) {
    // the stash pool word the place step tries first
    if (lane == 0) acc ^= pa.st_used[alloc_hash(pa.epoch, 0) % pa.PW];
  } else {
    // both bins of the remap pair: load, list, claim, removal mask, HBM page
    const uint2 rp = fa.rpair[0];
#pragma unroll
    for (uint32_t r = 0; r < 2; ++r) {
      const uint32_t b = r ? rp.y : rp.x;
      if (lane == 0) acc ^= fa.load[b] ^ fa.rev_cnt[b] ^ fa.claim[b] ^ fa.rmask[b];
      if (lane < 2 * fa.Z) acc ^= fa.rev_idx[(uint64_t)b * 2 * fa.Z + lane];
      if (b < fa.K && !fa.decomp)
        for (uint64_t w = lane; w < fa.pw; w += 64) acc ^= fa.hbm[(uint64_t)b * fa.pw + w];
    }
  }
  if (acc == 0x5D1F0C9B7A3E6421ull) set_err(fa.ctlw, 0);
}

__global__ __launch_bounds__(kSoloNT) void k_acc_solo(GroupArgs gr, FetchArgs fa, ResolveArgs rv, PlaceArgs pa,
                                                      WbArgs wa, FinishArgs fn, uint32_t wb_stride) {
  extern __shared__ uint64_t sdyn[];
  const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (threadIdx.x == 0) {
    // the command leads its key; a PUT or DEL is its key's last write
    const uint8_t op = gr.ops[0];
    gr.leader[0] = 0;
    gr.prevw[0] = kNone;
    gr.lastw[0] = (op & 3u) ? 0 : kNone;
    if (op > 2) gr.ctl->reject = gr.epoch;
  }
  if (lane == 0 && wave >= 1) group_prf(gr, wave - 1);
  if (fa.tlog_r && threadIdx.x < 5) fa.tlog_r[threadIdx.x] = kNone;  // the batch's trace words
  solo_step();
  if (wave == 0)
    fetch_cmd<false, true>(fa, 0, nullptr);
  else
    solo_warm(fa, pa, wave, lane);
  solo_step();
  if (wave == 0) {  // resolve and place in the same thread
    Settled st;
    resolve_cmd(rv, lane, &st);
    place_cmd(pa, lane, &st);
  }
  solo_step();
  compose_slot<false>(wa, wave, sdyn + (uint64_t)wave * (wb_stride / 8));
  solo_step();
  // the insert and the counters; the rebuild of slot s adds to bucket s only
  if (threadIdx.x == 0 && fn.ctl->reject != fn.epoch) {
    const bool ok = !fn.ctl->err;
    if (ok) finish_cmd(fn, 0);
    const uint64_t freed = (uint64_t)fn.freed[0] + fn.freed[1] + fn.freed[2];
    fn.freed[0] = 0;
    fn.freed[1] = 0;
    fn.freed[2] = 0;
    if (fn.decomp) {  // the three slots' staged frees go to the ring
      uint32_t give = 0;
      for (uint32_t s = 0; s < 3; ++s)
        for (uint32_t j = 0; j < fn.rfree_n[s]; ++j)
          fn.ring[(fn.ctl->ring_tail + give++) % fn.P] = fn.rfree[(uint64_t)s * fn.Z2 + j];
      fn.ctl->ring_give = give;
    }
    finish_apply(fn, ok, freed);
  }
}

// Fill of the trace segment of a batch (no memset nodes in captured graphs).
__global__ void k_fill_u32(uint32_t* p, uint64_t n, uint32_t v) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------

// The send of the outbox slots [lo, hi) of the map's last batch.
static ShipArgs ship_args(bolt_map* m, uint32_t lo, uint32_t hi) {
  ShipArgs a;
  a.ctl = m->ctl;
  a.lo = lo;
  a.hi = hi;
  a.pw = m->s.page_bytes / 8;
  a.ship_page = m->bs.ship_page + (uint64_t)m->ship_half * 2 * kMaxBatch;
  a.outbox = reinterpret_cast<const uint64_t*>(m->bs.outbox) + (uint64_t)m->ship_half * 2 * kMaxBatch * a.pw;
  a.obs = reinterpret_cast<uint64_t*>(m->obs);
  a.tags = reinterpret_cast<uint64_t*>(m->tags);
  a.pver = m->pver;
  return a;
}

// Fills every kernel argument of one map's batch; reserves its trace words.
static void plan_access(bolt_map* m, const uint8_t* ops, const uint64_t* keys, const void* vals_in, void* vals_out,
                        uint8_t* status, uint32_t q, hipStream_t st, AccessPlan& P, bool fill_trace = true) {
  const Sizes& s = m->s;
  const BatchScratch& bs = m->bs;
  const uint32_t epoch = (uint32_t)(m->batches + 1);
  const bool fast = q <= (s.B + 15) / 16 && q <= (s.R + 15) / 16;
  uint32_t* tlog_r = nullptr;
  uint32_t* tlog_w = nullptr;
  if (m->tlog) {
    const uint64_t words = 5ull * q;
    if (m->tlog_used + words <= m->tlog_cap) {
      tlog_r = m->tlog + m->tlog_used;
      tlog_w = tlog_r + 2ull * q;
      TraceSeg g{epoch, m->tlog_used, 2ull * q, 3ull * q};
      m->segs.push_back(g);
      m->tlog_used += words;
      if (fill_trace)
        hipLaunchKernelGGL(k_fill_u32, dim3((uint32_t)((words + 255) / 256)), dim3(256), 0, st, tlog_r, words, kNone);
    } else {
      m->tlog_lost = true;
    }
  }
  memset(&P, 0, sizeof(P));
  P.q = q;
  P.fast = fast ? 1 : 0;
  P.wb_lds = wb_lds_bytes(s.page_bytes / 8) + (m->tags ? s.page_bytes : 0);
  P.fetch_lds = m->tags ? 4 * s.page_bytes : 0;
  const uint32_t vw = s.vs / 8;
  const uint64_t* vin = reinterpret_cast<const uint64_t*>(vals_in);
  const uint64_t* fval = reinterpret_cast<const uint64_t*>(bs.fval);

  P.gr = GroupArgs{ops, keys, q, epoch, s.B, s.R, m->ctl, bs.leader, bs.prevw, bs.lastw, bs.fpair, bs.rpair, bs.rows};

  FetchArgs& fa = P.fa;
  fa.ctl = m->ctl;
  fa.ops = ops;
  fa.keys = keys;
  fa.leader = bs.leader;
  fa.fpair = bs.fpair;
  fa.rows = bs.rows;
  fa.q = q;
  fa.epoch = epoch;
  fa.B = s.B;
  fa.K = s.K;
  fa.R = s.R;
  fa.Z = (uint32_t)s.Z;
  fa.W = (uint32_t)s.W;
  fa.d = (uint32_t)s.d;
  fa.vw = vw;
  fa.pw = s.page_bytes / 8;
  fa.pm_key = m->pm_key;
  fa.pm_pair = m->pm_pair;
  fa.pm_mask = m->pm_mask;
  fa.obs = reinterpret_cast<const uint64_t*>(m->obs);
  fa.hbm = reinterpret_cast<const uint64_t*>(m->hbm);
  fa.rev_cnt = m->rev_cnt;
  fa.rev_idx = m->rev_idx;
  fa.st_key = m->st_key;
  fa.st_val = reinterpret_cast<const uint64_t*>(m->st_val);
  fa.st_dead = m->st_dead;
  fa.load = m->load;
  fa.load0 = m->load0;
  fa.fast = fast ? 1 : 0;
  fa.lastw = bs.lastw;
  fa.pm_mask_w = m->pm_mask;
  fa.claim = m->claim;
  fa.rmask = m->rmask;
  fa.stage = reinterpret_cast<uint64_t*>(bs.stage);
  fa.cand_bin = bs.cand_bin;
  fa.hit = bs.hit;
  fa.hrow = bs.hrow;
  fa.hslot = bs.hslot;
  fa.found = bs.found;
  fa.fval = reinterpret_cast<uint64_t*>(bs.fval);
  fa.rpair = bs.rpair;
  fa.tlog_r = tlog_r;
  fa.ctlw = m->ctl;
  fa.tags = reinterpret_cast<const uint64_t*>(m->tags);
  fa.pver = m->pver;
  fa.wslot = m->wslot;
  // the previous batch's half of the outbox (the pages it rebuilt)
  fa.outbox = reinterpret_cast<const uint64_t*>(bs.outbox) + (uint64_t)((epoch - 1) & 1) * 2 * kMaxBatch * fa.pw;
  fa.ov_epoch = m->ov_off ? 0 : epoch - 1;
  m->ov_off = false;
  fa.pre_host = m->obs_host ? 0 : 1;
  const uint32_t decomp = (m->p.flags & BOLT_F_DECOMPOSED) ? 1 : 0;
  fa.decomp = decomp;
  fa.ship = ship_args(m, 0, 0);  // run_access hands slices of the previous batch's send to its kernels
  fa.ship_blocks = 0;
  P.gr.ship = fa.ship;
  P.gr.ship_blocks = 0;

  ResolveArgs& rv = P.rv;
  rv.ctl = m->ctl;
  rv.ship = ship_args(m, 0, 0);
  rv.ship_blocks = 0;
  rv.ops = ops;
  rv.vals_in = vin;
  rv.leader = bs.leader;
  rv.prevw = bs.prevw;
  rv.lastw = bs.lastw;
  rv.hit = bs.hit;
  rv.hrow = bs.hrow;
  rv.hslot = bs.hslot;
  rv.found = bs.found;
  rv.fval = fval;
  rv.rpair = bs.rpair;
  rv.load = m->load0;  // the choice reads the loads as placement began
  rv.q = q;
  rv.vw = vw;
  rv.fast = P.fast;
  rv.epoch = epoch;
  rv.vals_out = reinterpret_cast<uint64_t*>(vals_out);
  rv.status = status;
  rv.fin = bs.fin;
  rv.chosen = bs.chosen;

  PlaceArgs& pa = P.pa;
  pa.several = !P.fast;
  pa.ctl = m->ctl;
  pa.ship = ship_args(m, 0, 0);
  pa.ship_blocks = 0;
  pa.keys = keys;
  pa.vals_in = vin;
  pa.leader = bs.leader;
  pa.lastw = bs.lastw;
  pa.fin = bs.fin;
  pa.chosen = bs.chosen;
  pa.hrow = bs.hrow;
  pa.hslot = bs.hslot;
  pa.fval = fval;
  pa.rpair = bs.rpair;
  pa.q = q;
  pa.epoch = epoch;
  pa.Z = (uint32_t)s.Z;
  pa.W = (uint32_t)s.W;
  pa.d = (uint32_t)s.d;
  pa.vw = vw;
  pa.K = s.K;
  pa.R = s.R;
  pa.PW = s.PW;
  pa.load = m->load;
  pa.st_used = m->st_used;
  pa.st_key = m->st_key;
  pa.st_val = reinterpret_cast<uint64_t*>(m->st_val);
  pa.st_dest = m->st_dest;
  pa.st_dead = m->st_dead;
  pa.rev_cnt = m->rev_cnt;
  pa.rev_idx = m->rev_idx;
  pa.claim = m->claim;
  pa.cand_bin = bs.cand_bin;
  pa.pm_pair = m->pm_pair;
  pa.pm_mask = m->pm_mask;
  pa.rowsel = bs.rowsel;
  pa.rows = bs.rows;
  pa.decomp = decomp;
  pa.ring = m->ring;
  pa.P = s.P;

  RemapArgs& ra = P.ra;
  ra.enabled = !P.fast;
  ra.ctl = m->ctl;
  ra.chosen = bs.chosen;
  ra.keys = keys;
  ra.vals_in = vin;
  ra.leader = bs.leader;
  ra.lastw = bs.lastw;
  ra.fin = bs.fin;
  ra.hrow = bs.hrow;
  ra.hslot = bs.hslot;
  ra.fval = fval;
  ra.rpair = bs.rpair;
  ra.q = q;
  ra.epoch = epoch;
  ra.Z = (uint32_t)s.Z;
  ra.W = (uint32_t)s.W;
  ra.d = (uint32_t)s.d;
  ra.vw = vw;
  ra.B = s.B;
  ra.K = s.K;
  ra.R = s.R;
  ra.PW = s.PW;
  ra.load = m->load;
  ra.st_used = m->st_used;
  ra.st_key = m->st_key;
  ra.st_val = reinterpret_cast<uint64_t*>(m->st_val);
  ra.st_dest = m->st_dest;
  ra.st_dead = m->st_dead;
  ra.rev_cnt = m->rev_cnt;
  ra.rev_idx = m->rev_idx;
  ra.claim = m->claim;
  ra.cand_bin = bs.cand_bin;
  ra.pm_key = m->pm_key;
  ra.pm_pair = m->pm_pair;
  ra.pm_mask = m->pm_mask;
  ra.rows = bs.rows;
  ra.decomp = decomp;
  ra.ring = m->ring;
  ra.P = s.P;

  WbArgs& wa = P.wa;
  wa.ctl = m->ctl;
  wa.q = q;
  wa.epoch = epoch;
  wa.Z = (uint32_t)s.Z;
  wa.vw = vw;
  wa.K = s.K;
  wa.pw = s.page_bytes / 8;
  wa.cand_bin = bs.cand_bin;
  wa.leader = bs.leader;
  wa.fin = bs.fin;
  wa.chosen = bs.chosen;
  wa.load = m->load;
  wa.load0 = m->load0;
  wa.claim = m->claim;
  wa.rmask = m->rmask;
  wa.stage = reinterpret_cast<const uint64_t*>(bs.stage);
  wa.hbm = reinterpret_cast<uint64_t*>(m->hbm);
  wa.rev_cnt = m->rev_cnt;
  wa.rev_idx = m->rev_idx;
  wa.st_key = m->st_key;
  wa.st_val = reinterpret_cast<const uint64_t*>(m->st_val);
  wa.st_dead = m->st_dead;
  wa.st_used = m->st_used;
  wa.freed = bs.freed;
  wa.tlog_w = tlog_w;
  wa.outbox = reinterpret_cast<uint64_t*>(bs.outbox) + (uint64_t)(epoch & 1) * 2 * kMaxBatch * (s.page_bytes / 8);
  wa.ship_page = bs.ship_page + (uint64_t)(epoch & 1) * 2 * kMaxBatch;
  wa.ship = ship_args(m, 0, 0);  // run_access hands it a slice of the previous batch's send
  wa.ship_blocks = 0;
  wa.wslot = m->wslot;
  wa.direct = 1;  // run_access switches a large host-store batch to the send
  wa.obs = reinterpret_cast<uint64_t*>(m->obs);
  wa.tags = reinterpret_cast<uint64_t*>(m->tags);
  wa.pver = m->pver;
  wa.decomp = decomp;
  wa.rfree = bs.rfree;
  wa.rfree_n = bs.rfree_n;


  FinishArgs& fn = P.fn;
  fn.ctl = m->ctl;
  fn.ship = ship_args(m, 0, 0);
  fn.ship_blocks = 0;
  fn.q = q;
  fn.W = (uint32_t)s.W;
  fn.epoch = epoch;
  fn.cap = s.cap;
  fn.stash_bound = s.stash_bound;
  fn.hbm_bound = decomp ? s.hbm_bound : ~0ull;
  fn.decomp = decomp;
  fn.Z2 = (uint32_t)(2 * s.Z);
  fn.ring = m->ring;
  fn.P = s.P;
  fn.rfree = bs.rfree;
  fn.rfree_n = bs.rfree_n;
  fn.rowsel = fast ? bs.rowsel : nullptr;
  fn.keys = keys;
  fn.rpair = bs.rpair;
  fn.freed = bs.freed;
  fn.pm_key = m->pm_key;
  fn.pm_pair = m->pm_pair;
  fn.pm_mask = m->pm_mask;
  m->batches++;
}

// BOLT_F_WATCH: the largest bin load and the items in the K HBM bins at the
// end of a batch, with their high-water marks (one workgroup).
__global__ __launch_bounds__(1024) void k_acc_watch(const uint32_t* __restrict__ load, uint64_t B, uint64_t K,
                                                    Ctl* ctl) {
  __shared__ uint32_t smax[16];
  __shared__ uint64_t ssum[16];
  uint32_t mx = 0;
  uint64_t sum = 0;
  for (uint64_t b = threadIdx.x; b < B; b += 1024) {
    const uint32_t l = load[b];
    mx = l > mx ? l : mx;
    sum += b < K ? l : 0;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const uint32_t om = __shfl_xor(mx, off, 64);
    mx = om > mx ? om : mx;
    sum += __shfl_xor(sum, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    smax[threadIdx.x >> 6] = mx;
    ssum[threadIdx.x >> 6] = sum;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 16; ++w) {
      mx = smax[w] > mx ? smax[w] : mx;
      sum += ssum[w];
    }
    if (mx > ctl->load_hw) ctl->load_hw = mx;
    ctl->hbm_load = sum;
    if (sum > ctl->hbm_hw) ctl->hbm_hw = sum;
  }
}

// The access pipeline for up to qmax commands of the maps of a device plan
// table (count of them), every phase one launch.
static void allow_big_lds();

// The bins of the map's loads that the several-round remap keeps in LDS
// (its dynamic LDS is 4 bytes a bin): all of them, or none.
static uint32_t remap_lds_bins(const bolt_map* m) { return m->s.B <= kRemapLdsBins ? (uint32_t)m->s.B : 0; }

static void launch_many(const AccessPlan& p0, const AccessPlan* tab, uint32_t C, uint32_t qmax, uint64_t lds,
                        uint64_t fetch_lds, bool any_slow, uint32_t remap_bins, hipStream_t st,
                        uint32_t ship_max = 0) {
  allow_big_lds();
  hipLaunchKernelGGL(k_acc_group<true>, dim3(kParts + group_prf_blocks(qmax), C), dim3(kDedupNT),
                     group_lds_bytes(qmax), st, p0.gr, tab);
  // each map's first ship_blocks workgroups of the fetch send its previous batch's pages
  const dim3 fgrid(ship_max + (qmax + 3) / 4, C);
  if (fetch_lds)  // a sealed map among them
    hipLaunchKernelGGL((k_acc_fetch<true, true>), fgrid, dim3(256), fetch_lds, st, p0.fa, tab);
  else
    hipLaunchKernelGGL((k_acc_fetch<true, false>), fgrid, dim3(256), 0, st, p0.fa, tab);
  hipLaunchKernelGGL(k_acc_resolve<true>, dim3((qmax + 63) / 64, C), dim3(64), 0, st, p0.rv, tab);
  if (any_slow)
    hipLaunchKernelGGL(k_acc_remap<true>, dim3(1, C), dim3(kRemapNT), 4ull * remap_bins, st, p0.ra, tab, 0u,
                       remap_bins);
  hipLaunchKernelGGL(k_acc_place<true>, dim3((qmax + 63) / 64, C), dim3(64), 0, st, p0.pa, tab);
  if (any_slow) hipLaunchKernelGGL(k_acc_remap<true>, dim3(1, C), dim3(kRemapNT), 0, st, p0.ra, tab, 1u, 0u);
  if (fetch_lds)  // a sealed map among them
    hipLaunchKernelGGL((k_acc_compose<true, true>), dim3(3 * qmax, C), dim3(64), lds, st, p0.wa, tab);
  else
    hipLaunchKernelGGL((k_acc_compose<true, false>), dim3(3 * qmax, C), dim3(64), lds, st, p0.wa, tab);
  hipLaunchKernelGGL(k_acc_finish<true>, dim3((qmax + 255) / 256, C), dim3(256), 0, st, p0.fn, tab);
}

// The dedup kernel's dynamic LDS reaches 96 KiB for the largest batches,
// the several-round remap's 96 KiB for the largest maps it keeps in LDS.
static void allow_big_lds() {
  static std::once_flag once;
  std::call_once(once, [] {
    const int bytes = (int)group_lds_bytes(kMaxBatch);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_acc_group<false>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_acc_group<true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    const int rbytes = (int)(4 * kRemapLdsBins);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_acc_remap<false>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, rbytes);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_acc_remap<true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, rbytes);
  });
}

// Smallest batch whose observable pages are sent during the next batch.
constexpr uint32_t kDeferMinBatch = 256;

// Shares (in 64ths of a batch's outbox slots) of the send carried by the
// batch's own finish and by the next batch's dedup, resolve, place and
// rebuild kernels.  The link is busy through the whole batch, so a slice
// only pays while it does not lengthen its kernel; these shares measured
// best (4096-command batches, 1 KiB pages: doubling them, or halving them
// again, was slower).  The next fetch carries the rest.  The next rebuild
// writes the other half of the outbox.  Sealed maps send from the fetch
// only (the send needs LDS there).
constexpr uint32_t kShareFinish = 1, kShareGroup = 2, kShareResolve = 1, kSharePlace = 3, kShareCompose = 6;
constexpr uint32_t kShipComposeWaves = 256;  // waves of the rebuild launch that send

int flush_ship(bolt_map* m, hipStream_t st) {
  if (!m->ship_q) return BOLT_OK;
  const ShipArgs a = ship_args(m, m->ship_from, 2 * m->ship_q);
  m->ship_q = 0;
  m->ship_from = 0;
  if (a.lo >= a.hi) return BOLT_OK;
  {
    TimedScope ts(m->timer, kkAccShip, st);
    hipLaunchKernelGGL(k_acc_ship, dim3(ship_blocks_for(a.hi - a.lo)), dim3(256), m->tags ? 4 * m->s.page_bytes : 0, st,
                       a);
  }
  return hipGetLastError() == hipSuccess ? BOLT_OK : BOLT_EHIP;
}

// One-map batch through a graph captured for its size class: the call's
// arguments go to the device plan, then the class's graph replays the
// pipeline (grids sized for the class; each kernel stops at the plan's q).
static int run_access_graph(bolt_map* m, AccessPlan& P, hipStream_t st) {
  uint32_t cls = 0;
  while ((1u << cls) < P.q) ++cls;
  if (!m->gplan) {
    if (hipMalloc(&m->gplan, sizeof(AccessPlan)) != hipSuccess) return BOLT_ENOMEM;
    m->allocs.push_back(m->gplan);
  }
  AccessPlan* tab = static_cast<AccessPlan*>(m->gplan);
  if (flush_ship(m, st)) return BOLT_EHIP;
  if (!m->gexec[cls]) {
    // the several-round kernels are in the graph too; the plan's flags say whether they run
    hipStream_t cs = m->side;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) return BOLT_EHIP;
    launch_many(P, tab, 1, 1u << cls, P.wb_lds, P.fetch_lds, true, remap_lds_bins(m), cs);
    if (hipStreamEndCapture(cs, &g) != hipSuccess || !g) return BOLT_EHIP;
    hipGraphExec_t ex = nullptr;
    const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return BOLT_EHIP;
    m->gexec[cls] = ex;
  }
  if (hipMemcpyAsync(tab, &P, sizeof(AccessPlan), hipMemcpyHostToDevice, st) != hipSuccess) return BOLT_EHIP;
  if (hipGraphLaunch(m->gexec[cls], st) != hipSuccess) return BOLT_EHIP;
  return BOLT_OK;
}

int run_access(bolt_map* m, const uint8_t* ops, const uint64_t* keys, const void* vals_in, void* vals_out,
               uint8_t* status, uint32_t q, hipStream_t st) {
  // A batch of one command on a plain map runs as one workgroup (k_acc_solo,
  // which also fills its trace words) when three rebuild waves' LDS fits
  // the default 64 KiB.  One command is always one round (B, R >= 1).
  const uint32_t wb_stride = (uint32_t)wb_lds_bytes(m->s.page_bytes / 8);
  const bool solo = q == 1 && !m->tags && !(m->p.flags & BOLT_F_GRAPHS) &&
                    3ull * wb_stride + 4 * kFreeBuckets <= 65536;
  AccessPlan P;
  plan_access(m, ops, keys, vals_in, vals_out, status, q, st, P, !solo);
  if (solo) {
    static_assert(sizeof(GroupArgs) + sizeof(FetchArgs) + sizeof(ResolveArgs) + sizeof(PlaceArgs) + sizeof(WbArgs) +
                          sizeof(FinishArgs) + 8 <= 4096,
                  "kernel arguments of k_acc_solo");
    if (flush_ship(m, st)) return BOLT_EHIP;
    P.wa.direct = 1;
    P.fa.pre_host = 1;  // no send shares the link: both pages are read at once
    {
      TimedScope ts(m->timer, kkAccSolo, st);
      hipLaunchKernelGGL(k_acc_solo, dim3(1), dim3(kSoloNT), 3ull * wb_stride, st, P.gr, P.fa, P.rv, P.pa, P.wa,
                         P.fn, wb_stride);
    }
    if (m->p.flags & BOLT_F_WATCH)
      hipLaunchKernelGGL(k_acc_watch, dim3(1), dim3(1024), 0, st, m->load, m->s.B, m->s.K, m->ctl);
    return hipGetLastError() == hipSuccess ? BOLT_OK : BOLT_EHIP;
  }
  if (m->p.flags & BOLT_F_GRAPHS) {
    const int rc = run_access_graph(m, P, st);
    if (rc == BOLT_OK && (m->p.flags & BOLT_F_WATCH))
      hipLaunchKernelGGL(k_acc_watch, dim3(1), dim3(1024), 0, st, m->load, m->s.B, m->s.K, m->ctl);
    return rc;
  }
  const AccessPlan* none = nullptr;
  allow_big_lds();
  // A large batch on a pinned host store rebuilds its observable pages into
  // its half of the outbox, and the next batch's kernels (or a flush) send
  // them.  Small batches and device stores, with no link time to hide, write
  // them from the rebuild.
  const bool defer = m->obs_host && q >= kDeferMinBatch;
  // The previous batch's rebuilt pages still to be sent, in slices: plain
  // maps spread them over this batch's dedup, resolve and place kernels
  // (each running anyway), the fetch takes the rest (writes over the link
  // while it reads).
  {
    const uint32_t end = 2 * m->ship_q;
    uint32_t lo = m->ship_from < end ? m->ship_from : end;
    auto take = [&](uint32_t share, ShipArgs& a, uint32_t& blocks, uint32_t waves_per_block, uint32_t max_waves) {
      const uint32_t n = end * share / 64, hi = lo + n < end ? lo + n : end;
      a = ship_args(m, lo, hi);
      blocks = (hi - lo + waves_per_block - 1) / waves_per_block;
      if (blocks > max_waves / waves_per_block) blocks = max_waves / waves_per_block;
      lo = hi;
    };
    if (end && !m->tags) {
      take(kShareGroup, P.gr.ship, P.gr.ship_blocks, kDedupNT / 64, 4 * kShipMaxBlocks);
      if (P.fast)  // resolve and place are one launch
        take(kShareResolve + kSharePlace, P.pa.ship, P.pa.ship_blocks, 1, 4 * kShipMaxBlocks);
      else
        take(kShareResolve, P.rv.ship, P.rv.ship_blocks, 1, 4 * kShipMaxBlocks);
      // The rebuild's one-wave workgroups, a few slots per wave (its own
      // waves already fill the device); only when this batch rebuilds into
      // the outbox: a rebuild that writes the store itself could race the
      // slice on a page both write.
      if (defer) take(kShareCompose, P.wa.ship, P.wa.ship_blocks, 1, kShipComposeWaves);
    }
    P.fa.ship = ship_args(m, lo, end);
    P.fa.ship_blocks = ship_blocks_for(end - lo);
    m->ship_q = 0;
    m->ship_from = 0;
  }
  {
    TimedScope ts(m->timer, kkAccDedup, st);
    hipLaunchKernelGGL(k_acc_group<false>, dim3(P.gr.ship_blocks + kParts + group_prf_blocks(q)), dim3(kDedupNT),
                       group_lds_bytes(q), st, P.gr, none);
  }
  {
    TimedScope ts(m->timer, kkAccFetch, st);
    const dim3 grid(P.fa.ship_blocks + (q + 3) / 4);
    if (P.fetch_lds)
      hipLaunchKernelGGL((k_acc_fetch<false, true>), grid, dim3(256), P.fetch_lds, st, P.fa, none);
    else
      hipLaunchKernelGGL((k_acc_fetch<false, false>), grid, dim3(256), 0, st, P.fa, none);
  }
  if (P.fast) {
    TimedScope ts(m->timer, kkAccRemap, st);
    hipLaunchKernelGGL(k_acc_settle, dim3(P.pa.ship_blocks + (q + 63) / 64), dim3(64), 0, st, P.rv, P.pa);
  } else {
    {
      TimedScope ts(m->timer, kkAccResolve, st);
      hipLaunchKernelGGL(k_acc_resolve<false>, dim3(P.rv.ship_blocks + (q + 63) / 64), dim3(64), 0, st, P.rv, none);
    }
    TimedScope ts(m->timer, kkAccRemap, st);
    hipLaunchKernelGGL(k_acc_remap<false>, dim3(1), dim3(kRemapNT), 4ull * remap_lds_bins(m), st, P.ra, none, 0u,
                       remap_lds_bins(m));
    hipLaunchKernelGGL(k_acc_place<false>, dim3(P.pa.ship_blocks + (q + 63) / 64), dim3(64), 0, st, P.pa, none);
    hipLaunchKernelGGL(k_acc_remap<false>, dim3(1), dim3(kRemapNT), 0, st, P.ra, none, 1u, 0u);
  }
  P.wa.direct = defer ? 0 : 1;
  {
    TimedScope ts(m->timer, kkAccCompose, st);
    if (m->tags)
      hipLaunchKernelGGL((k_acc_compose<false, true>), dim3(3 * q), dim3(64), P.wb_lds, st, P.wa, none);
    else
      hipLaunchKernelGGL((k_acc_compose<false, false>), dim3(P.wa.ship_blocks + 3 * q), dim3(64), P.wb_lds, st,
                         P.wa, none);
  }
  m->ship_q = defer ? q : 0;
  m->ship_from = 0;
  m->ship_half = P.fa.epoch & 1;  // the half this batch rebuilt its pages into
  if (defer && !m->tags) {  // the finish starts this batch's send
    const uint32_t hi = 2 * q * kShareFinish / 64;
    P.fn.ship = ship_args(m, 0, hi);
    P.fn.ship_blocks = ship_blocks_for(hi);
    m->ship_from = hi;
  }
  {
    TimedScope ts(m->timer, kkAccMisc, st);
    hipLaunchKernelGGL(k_acc_finish<false>, dim3(P.fn.ship_blocks + (q + 255) / 256), dim3(256), 0, st, P.fn, none);
  }
  if (m->p.flags & BOLT_F_WATCH)
    hipLaunchKernelGGL(k_acc_watch, dim3(1), dim3(1024), 0, st, m->load, m->s.B, m->s.K, m->ctl);
  return hipGetLastError() == hipSuccess ? BOLT_OK : BOLT_EHIP;
}

// One batch for each of `count` distinct maps, every phase one launch for
// all of them (map = blockIdx.y).  The plans go to the device in one copy.
int run_access_many(bolt_map* const* maps, const bolt_batch* batches, uint32_t count, hipStream_t st,
                    bool defer_pages) {
  std::vector<AccessPlan> plans(count);
  uint32_t qmax = 0, ship_max = 0;
  uint64_t lds = 0, flds = 0;
  bool any_slow = false;
  uint32_t remap_bins = 0;
  std::vector<uint8_t> defer(count, 0);
  for (uint32_t i = 0; i < count; ++i) {
    const bolt_batch& b = batches[i];
    bolt_map* m = maps[i];
    // The map's previous batch's pages still to be sent go out from this
    // launch's fetch, beside its reads (as in one-map batches).
    ShipArgs pending = ship_args(m, m->ship_from, 2 * m->ship_q);
    const bool has_pending = m->ship_q && m->ship_from < 2 * m->ship_q;
    m->ship_q = 0;
    m->ship_from = 0;
    plan_access(m, b.d_ops, b.d_keys, b.d_vals_in, b.d_vals_out, b.d_status, b.q, st, plans[i]);
    if (has_pending) {
      plans[i].fa.ship = pending;
      plans[i].fa.ship_blocks = ship_blocks_for(pending.hi - pending.lo);
      ship_max = plans[i].fa.ship_blocks > ship_max ? plans[i].fa.ship_blocks : ship_max;
    }
    // a large batch on a pinned store rebuilds its pages into its outbox half,
    // when the caller runs more batches of these maps soon (serving)
    defer[i] = defer_pages && m->obs_host && b.q >= kDeferMinBatch;
    plans[i].wa.direct = defer[i] ? 0 : 1;
    qmax = b.q > qmax ? b.q : qmax;
    lds = plans[i].wb_lds > lds ? plans[i].wb_lds : lds;
    flds = plans[i].fetch_lds > flds ? plans[i].fetch_lds : flds;
    any_slow |= plans[i].fast == 0;
    if (!plans[i].fast) remap_bins = std::max(remap_bins, remap_lds_bins(m));
  }
  AccessPlan* tab = nullptr;
  const size_t bytes = sizeof(AccessPlan) * count;
  if (hipMallocAsync((void**)&tab, bytes, st) != hipSuccess) return BOLT_ENOMEM;
  if (hipMemcpyAsync(tab, plans.data(), bytes, hipMemcpyHostToDevice, st) != hipSuccess) {
    (void)hipFreeAsync(tab, st);
    return BOLT_EHIP;
  }
  launch_many(plans[0], tab, count, qmax, lds, flds, any_slow, remap_bins, st, ship_max);
  for (uint32_t i = 0; i < count; ++i) {
    maps[i]->ship_q = defer[i] ? batches[i].q : 0;
    maps[i]->ship_from = 0;
    maps[i]->ship_half = plans[i].fa.epoch & 1;  // the half this batch rebuilt its pages into
  }
  for (uint32_t i = 0; i < count; ++i)
    if (maps[i]->p.flags & BOLT_F_WATCH)
      hipLaunchKernelGGL(k_acc_watch, dim3(1), dim3(1024), 0, st, maps[i]->load, maps[i]->s.B, maps[i]->s.K,
                         maps[i]->ctl);
  (void)hipFreeAsync(tab, st);
  return hipGetLastError() == hipSuccess ? BOLT_OK : BOLT_EHIP;
}

}  // namespace bolt
