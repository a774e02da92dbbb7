// Oblivious build of the map (the "fast data initialization" of Sec. 5.2,
// done on the device without a trusted data owner).
//
//   a1  PRF: each key gets two distinct bins (Sec. 4.1).
//   a2  P2C: each key goes to the less loaded of its bins, in rounds of
//       ceil(B/16) keys that see the loads at the start of their round.
//   a3  Bitonic sort of (bin << 32 | input index) tags.
//   a4  Rank inside the bin -> target slot bin * Z + rank.
//   a5  Expansion network into B * Z dummy-padded slots.
//   a6  Write-out: every bin as a canonical page (items sorted by key);
//       HBM bins, then observable pages 0..M-1, whole pages.
//   a7  Position map: key -> (p1, p2) in the least loaded of d rows
//       (Sec. 5.2), in rounds of ceil(R/16) keys; then a duplicate check.
//
// Grid shapes and trip counts depend only on n and the map's sizes.
#include <string.h>

#include <algorithm>
#include <vector>

#include "bolt_impl.h"
#include "seal_dev.h"

namespace bolt {

// ---------------------------------------------------------------------------
// wave / block scans
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  const uint32_t lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    uint32_t y = __shfl_up(x, off, 64);
    if (lane >= (uint32_t)off) x += y;
  }
  return x;
}

// Exclusive scan of one value per thread over the block; *total (shared)
// gets the block sum.  Every thread of the block must call it.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t* total) {
  __shared__ uint32_t wsum[NT / 64];
  const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint32_t inc = wave_incl_scan(x);
  if (lane == 63) wsum[wid] = inc;
  __syncthreads();
  if (wid == 0) {
    uint32_t v = lane < NT / 64 ? wsum[lane] : 0;
    uint32_t vi = wave_incl_scan(v);
    if (lane < NT / 64) wsum[lane] = vi - v;
    if (lane == NT / 64 - 1) *total = vi;
  }
  __syncthreads();
  const uint32_t r = wsum[wid] + inc - x;
  __syncthreads();
  return r;
}

constexpr int kScanNT = 256;
constexpr int kScanPer = 16;
constexpr uint32_t kScanChunk = kScanNT * kScanPer;

// Everything one map's build needs on the device: its sizes, state, inputs
// and scratch.  A many-map launch reads the plan of map blockIdx.y from a
// table; a one-map launch takes it by value.
struct BuildPlan {
  Ctl* ctl;
  const uint64_t* keys;
  const uint64_t* vals;
  uint64_t n, npad, B, K, BZ, R, pw;
  uint64_t rs, rsm;  // keys per P2C round, keys per position-map round
  uint32_t Z, vw, W, d, nbs;
  uint64_t* hbm;
  uint64_t* obs;
  uint32_t* tlog;  // write-out trace (M words) or null
  uint64_t* tags;  // BOLT_F_SEAL: [M][2] page tags (observable), else null
  uint64_t* pver;  // BOLT_F_SEAL: [M] page write counts
  uint32_t* load;
  uint32_t* load0;  // the copy the access path's placement reads
  uint64_t* pm_key;
  uint2* pm_pair;
  uint32_t* pm_mask;
  // BOLT_F_DECOMPOSED: the HBM bins' items go to the value pool, listed
  // under their bin, and the pool's free-address ring starts after them
  uint32_t decomp;
  uint64_t pool, hbm_bound;
  uint32_t* ring;
  uint64_t* st_key;
  uint64_t* st_val;
  uint32_t* st_dest;
  uint32_t* st_dead;
  uint32_t* rev_cnt;
  uint32_t* rev_idx;
  // scratch
  uint2* pair;      // [n]
  uint32_t* dest;   // [n]
  uint64_t* tag;    // [npad]
  uint64_t* elem;   // [BZ]
  uint64_t* tmp;    // [BZ]
  uint32_t* start;  // [B] first sorted position of each bin
  uint32_t* bsum;   // [nbs + 1] scan partials, then the max-key counter
  uint64_t* rstate; // [R] row fill word of the position-map rounds
};

#define BOLT_PLAN const BuildPlan& P = MULTI ? tab[blockIdx.y] : p1
#define BOLT_PLAN_ARGS BuildPlan p1, const BuildPlan* tab

// Exclusive scan of the bin loads into the first sorted position of each bin.
template <bool MULTI>
__global__ __launch_bounds__(kScanNT) void k_scan_reduce(BOLT_PLAN_ARGS) {
  BOLT_PLAN;
  if (blockIdx.x >= P.nbs) return;  // whole block
  const uint64_t base = (uint64_t)blockIdx.x * kScanChunk + (uint64_t)threadIdx.x * kScanPer;
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) s += base + i < P.B ? P.load[base + i] : 0;
  __shared__ uint32_t tot;
  block_excl_scan<kScanNT>(s, &tot);
  if (threadIdx.x == 0) P.bsum[blockIdx.x] = tot;
}

// Exclusive scan of the block sums in one block, chunk by chunk.
template <bool MULTI>
__global__ __launch_bounds__(kScanNT) void k_scan_top(BOLT_PLAN_ARGS) {
  BOLT_PLAN;
  __shared__ uint32_t tot;
  uint32_t carry = 0;
  for (uint32_t c = 0; c < P.nbs; c += kScanNT) {
    uint32_t i = c + threadIdx.x;
    uint32_t v = i < P.nbs ? P.bsum[i] : 0;
    uint32_t e = block_excl_scan<kScanNT>(v, &tot);
    __syncthreads();
    if (i < P.nbs) P.bsum[i] = carry + e;
    carry += tot;
    __syncthreads();
  }
}

template <bool MULTI>
__global__ __launch_bounds__(kScanNT) void k_scan_down(BOLT_PLAN_ARGS) {
  BOLT_PLAN;
  if (blockIdx.x >= P.nbs) return;  // whole block
  const uint64_t base = (uint64_t)blockIdx.x * kScanChunk + (uint64_t)threadIdx.x * kScanPer;
  uint32_t v[kScanPer];
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    v[i] = base + i < P.B ? P.load[base + i] : 0;
    s += v[i];
  }
  __shared__ uint32_t tot;
  uint32_t e = block_excl_scan<kScanNT>(s, &tot) + P.bsum[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    if (base + i < P.B) P.start[base + i] = e;
    e += v[i];
  }
}

// ---------------------------------------------------------------------------
// map init
// ---------------------------------------------------------------------------

// Pool bitmap: every entry free, the bits past the pool size set.
__global__ void k_pool_init(uint64_t* used, uint64_t P, uint64_t PW) {
  uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= PW) return;
  const uint64_t lo = w * 64;
  uint64_t v = 0;
  if (lo + 64 > P) v = ~0ull << (P - lo);  // P - lo in [1, 63] for the last word
  used[w] = v;
}

__global__ void k_ctl_init(Ctl* ctl) {
  if (threadIdx.x || blockIdx.x) return;
  ctl->err = 0;
  ctl->reject = 0;
  ctl->steps = 0;
  ctl->live = 0;
  ctl->stash_live = 0;
  ctl->stash_hw = 0;
  ctl->b_place = 0;
  ctl->b_ins = 0;
  ctl->b_del = 0;
  ctl->load_hw = 0;
  ctl->hbm_load = 0;
  ctl->hbm_hw = 0;
  ctl->seq = 0;
  ctl->ring_head = 0;
  ctl->ring_tail = 0;
  ctl->ring_take = 0;
  ctl->ring_give = 0;
  ctl->pool_live = 0;
  ctl->hbm_live = 0;
  ctl->b_hbm_in = 0;
  ctl->b_hbm_rm = 0;
  ctl->fin_done = 0;
  ctl->pad0 = 0;
}

void launch_map_init(bolt_map* m, hipStream_t st) {
  const Sizes& s = m->s;
  (void)hipMemsetAsync(m->load, 0, s.B * sizeof(uint32_t), st);
  (void)hipMemsetAsync(m->pm_mask, 0, s.R * sizeof(uint32_t), st);
  (void)hipMemsetAsync(m->rev_cnt, 0, s.B * sizeof(uint32_t), st);
  (void)hipMemsetAsync(m->claim, 0, s.B * sizeof(uint64_t), st);
  (void)hipMemsetAsync(m->rmask, 0, s.B * sizeof(uint64_t), st);
  (void)hipMemsetAsync(m->st_dead, 0, s.P * sizeof(uint32_t), st);
  hipLaunchKernelGGL(k_pool_init, dim3((uint32_t)((s.PW + 255) / 256)), dim3(256), 0, st, m->st_used, s.P, s.PW);
  hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, st, m->ctl);
  launch_prf_key_setup(m->ctl, m->p.key, st);
}

// ---------------------------------------------------------------------------
// a1 + a2
// ---------------------------------------------------------------------------

template <bool MULTI>
__global__ void k_build_pairs(BOLT_PLAN_ARGS) {
  BOLT_PLAN;
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P.n) return;
  uint32_t hk[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) hk[j] = P.ctl->hkey[j];
  uint64_t w[4];
  prf4(hk, kDomPair, P.keys[i], w);
  uint32_t a, b;
  pair_of(w[0], w[1], P.B, a, b);
  P.pair[i] = make_uint2(a, b);
}

// A row's count during the position-map rounds, as one 64-bit word updated
// with compare-and-swap: [last round that added : 16][count when that round
// began : 24][count now : 24].  A key of round r reads the count at the
// start of its round from either field, whether or not other keys of the
// round have already added, so one launch per round both decides and adds
// (rounds are numbered from 1; the word starts at zero).
constexpr uint64_t kCntMask = 0xFFFFFFull;

__device__ __forceinline__ uint32_t round_start_count(uint64_t w, uint32_t r) {
  return (uint32_t)((w >> 48) == r ? (w >> 24) & kCntMask : w & kCntMask);
}

// Adds one in round r; returns the count before (the new item's slot).
// `old` is a recent read of the word (a guess: a stale one costs a retry).
__device__ __forceinline__ uint32_t round_add(uint64_t* word, uint64_t old, uint32_t r, Ctl* ctl) {
  unsigned long long* p = reinterpret_cast<unsigned long long*>(word);
  while (true) {
    const uint64_t cur = old & kCntMask;
    if (cur == kCntMask) {  // saturated: far beyond any capacity
      set_err(ctl, kErrOverflow);
      return (uint32_t)cur;
    }
    const uint64_t base = (old >> 48) == r ? (old >> 24) & kCntMask : cur;
    const uint64_t nw = ((uint64_t)r << 48) | (base << 24) | (cur + 1);
    const uint64_t prev = atomicCAS(p, (unsigned long long)old, (unsigned long long)nw);
    if (prev == old) return (uint32_t)cur;
    old = prev;
  }
}

// One P2C round (numbered from 1) in two launches: every key of the round
// picks the less loaded of its two bins as loaded when the round began
// (ties to the first bin), then all of them add.  (A fused round with the
// round-tagged words above costs a compare-and-swap round trip per key,
// slower here than a fire-and-forget add plus one more launch.)
template <bool MULTI>
__global__ void k_p2c_decide(BOLT_PLAN_ARGS, uint32_t round) {
  BOLT_PLAN;
  const uint64_t r0 = (uint64_t)(round - 1) * P.rs, r1 = r0 + P.rs < P.n ? r0 + P.rs : P.n;
  uint64_t i = r0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= r1) return;
  const uint2 p = P.pair[i];
  P.dest[i] = P.load[p.y] < P.load[p.x] ? p.y : p.x;
}

template <bool MULTI>
__global__ void k_p2c_add(BOLT_PLAN_ARGS, uint32_t round) {
  BOLT_PLAN;
  const uint64_t r0 = (uint64_t)(round - 1) * P.rs, r1 = r0 + P.rs < P.n ? r0 + P.rs : P.n;
  uint64_t i = r0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= r1) return;
  atomicAdd(&P.load[P.dest[i]], 1u);
}

template <bool MULTI>
__global__ void k_check_loads(BOLT_PLAN_ARGS) {
  BOLT_PLAN;
  uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b < P.B) P.load0[b] = P.load[b];
  bool bad = b < P.B && P.load[b] > P.Z;
  if (__any(bad) && (threadIdx.x & 63) == 0) set_err(P.ctl, kErrOverflow);
}

// ---------------------------------------------------------------------------
// a3 + a4
// ---------------------------------------------------------------------------

template <bool MULTI>
__global__ void k_make_tags(BOLT_PLAN_ARGS) {
  BOLT_PLAN;
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P.npad) return;
  uint64_t b = i < P.n ? P.dest[i] : 0xFFFFFFFFull;
  P.tag[i] = (b << 32) | (uint32_t)i;
}

// Element for slot placement: (bin * Z + rank) << 32 | input index.
template <bool MULTI>
__global__ void k_make_elems(BOLT_PLAN_ARGS) {
  BOLT_PLAN;
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P.BZ) return;
  uint64_t e = kNone64;
  if (i < P.n) {
    uint64_t t = P.tag[i];
    uint32_t b = (uint32_t)(t >> 32);
    uint64_t rank = b < P.B ? i - P.start[b] : P.Z;
    if (rank < P.Z)
      e = (((uint64_t)b * P.Z + rank) << 32) | (uint32_t)t;
    else
      set_err(P.ctl, kErrOverflow);
  }
  P.elem[i] = e;
}

// ---------------------------------------------------------------------------
// a6: one wave per bin.  `flip`: the expansion result is in tmp, not elem.
// ---------------------------------------------------------------------------

template <bool MULTI>
__global__ __launch_bounds__(256) void k_writeout(BOLT_PLAN_ARGS, uint32_t flip) {
  BOLT_PLAN;
  __shared__ uint32_t by_rank[4][64];
  __shared__ uint64_t key_rank[4][64];
  const uint64_t* __restrict__ elem = flip ? P.tmp : P.elem;
  const uint32_t Z = P.Z, vw = P.vw;
  const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint64_t b = (uint64_t)blockIdx.x * 4 + wid;
  const bool active = b < P.B;  // no early return: the barrier below needs every wave
  uint32_t src = kNone;
  uint64_t key = 0;
  if (active && lane < Z) {
    uint64_t e = elem[b * Z + lane];
    if (e != kNone64) {
      src = (uint32_t)e;
      key = P.keys[src];
    }
  }
  const bool valid = src != kNone;
  const uint64_t vmask = __ballot(valid);
  const uint32_t cnt = __popcll(vmask);
  // rank by key among the real items; ranks are a permutation of [0, cnt)
  // even if a key repeats (duplicate build keys are reported, not trusted)
  uint32_t rank = 0;
  for (uint32_t j = 0; j < Z; ++j) {
    uint64_t kj = __shfl(key, j, 64);
    bool vj = (vmask >> j) & 1;
    rank += (vj && (kj < key || (kj == key && j < lane))) ? 1 : 0;  // lane order breaks ties
  }
  if (valid && rank < 64) {
    by_rank[wid][rank] = src;
    key_rank[wid][rank] = key;
  }
  __syncthreads();
  const uint64_t pw = P.pw;
  // word w of the bin's canonical page
  auto word = [&](uint64_t w) -> uint64_t {
    uint64_t v = 0;
    if (w == 0) {
      v = cnt >= 64 ? kNone64 : ((1ull << cnt) - 1);
    } else if (w <= Z) {
      uint32_t j = (uint32_t)w - 1;
      v = j < cnt ? key_rank[wid][j] : 0;
    } else if (w < 1 + Z + (uint64_t)Z * vw) {
      uint64_t off = w - 1 - Z;
      uint32_t j = (uint32_t)(off / vw), o = (uint32_t)(off % vw);
      v = j < cnt ? P.vals[(uint64_t)by_rank[wid][j] * vw + o] : 0;
    }
    return v;
  };
  // A decomposed store keeps an HBM bin's items as value-pool entries
  // start[b] + rank (the bins' loads scanned, so HBM bin b's items follow
  // those of bins 0..b-1), listed under the bin; it has no HBM pages.
  const bool pooled = P.decomp && b < P.K;  // the same for the whole wave
  auto pool_write = [&]() {
    for (uint32_t j = lane; j < cnt; j += 64) {
      const uint64_t e = (uint64_t)P.start[b] + j;
      if (e >= P.pool) {  // more items than the pool holds: reported, nothing written
        set_err(P.ctl, kErrOverflow);
        continue;
      }
      P.st_key[e] = key_rank[wid][j];
      for (uint32_t o = 0; o < vw; ++o) P.st_val[e * vw + o] = P.vals[(uint64_t)by_rank[wid][j] * vw + o];
      P.st_dest[e] = (uint32_t)b;
      P.st_dead[e] = 0;
      P.rev_idx[b * 2 * Z + j] = (uint32_t)e;
    }
    if (lane == 0) P.rev_cnt[b] = cnt;
  };
  uint64_t* dst = b < P.K ? (pooled ? nullptr : P.hbm + b * pw) : P.obs + (b - P.K) * pw;
  if (!P.tags) {  // unsealed map (the same for the whole block)
    if (!active) return;
    if (pooled) {
      pool_write();
      return;
    }
    for (uint64_t w = lane; w < pw; w += 64) dst[w] = word(w);
    if (P.tlog && b >= P.K && lane == 0) P.tlog[b - P.K] = (uint32_t)(b - P.K);
    return;
  }
  // Sealed map: an observable page is composed in LDS, encrypted there,
  // tagged, and written once (write count 1).  HBM bins stay plain.
  extern __shared__ uint64_t wdyn[];
  uint64_t* pg = wdyn + (uint64_t)wid * pw;
  const bool seal = active && b >= P.K;  // the same for the whole wave
  if (active) {
    if (seal)
      for (uint64_t w = lane; w < pw; w += 64) pg[w] = word(w);
    else if (pooled)
      pool_write();
    else
      for (uint64_t w = lane; w < pw; w += 64) dst[w] = word(w);
  }
  __syncthreads();
  uint32_t skey[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) skey[j] = P.ctl->skey[j];
  const uint32_t page = (uint32_t)(b - P.K);
  uint32_t ks[16], otk[8], tag[4];
  if (seal) {
    chacha_first_pass(skey, page, 1u, 0u, ks, otk);
    chacha_page_xor(pg, (uint32_t)pw, ks, skey, page, 1u, 0u);
  }
  __syncthreads();
  if (!seal) return;
  poly_page_tag(pg, (uint32_t)pw, otk, tag);
  for (uint64_t w = lane; w < pw; w += 64) dst[w] = pg[w];
  if (lane == 0) {
    P.tags[2 * (uint64_t)page] = (uint64_t)tag[0] | ((uint64_t)tag[1] << 32);
    P.tags[2 * (uint64_t)page + 1] = (uint64_t)tag[2] | ((uint64_t)tag[3] << 32);
    P.pver[page] = 1;
    if (P.tlog) P.tlog[page] = page;
  }
}

// ---------------------------------------------------------------------------
// a7: position map
// ---------------------------------------------------------------------------

__device__ __forceinline__ void pm_rows_of(const uint32_t hk[8], uint64_t key, uint64_t R, uint32_t d,
                                           uint32_t rows[4]) {
  uint64_t w[4];
  prf4(hk, kDomRows, key, w);
#pragma unroll
  for (int j = 0; j < 4; ++j) rows[j] = (uint32_t)__umul64hi(w[j], R);
  for (uint32_t j = d; j < 4; ++j) rows[j] = rows[0];
}

// Row counters and the max-key counter start at zero (a kernel, not a
// memset, so the sequence can be captured in a graph).
template <bool MULTI>
__global__ void k_build_zero(BOLT_PLAN_ARGS) {
  BOLT_PLAN;
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < P.R) P.rstate[i] = 0;
  if (i < P.B) P.load[i] = 0;
  if (i == 0) P.bsum[P.nbs] = 0;
}

// One position-map round (numbered from 1): each key goes to the least
// filled of its d rows as filled when the round began (ties to the first),
// into the next free slot.
template <bool MULTI>
__global__ void k_pm_round(BOLT_PLAN_ARGS, uint32_t round) {
  BOLT_PLAN;
  const uint64_t r0 = (uint64_t)(round - 1) * P.rsm, r1 = r0 + P.rsm < P.n ? r0 + P.rsm : P.n;
  uint64_t i = r0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= r1) return;
  uint32_t hk[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) hk[j] = P.ctl->hkey[j];
  const uint64_t key = P.keys[i];
  uint32_t rows[4];
  pm_rows_of(hk, key, P.R, P.d, rows);
  uint32_t best = rows[0];
  uint64_t bw = P.rstate[rows[0]];  // plain loads, as in the P2C round
  uint32_t bc = round_start_count(bw, round);
  for (uint32_t j = 1; j < P.d; ++j) {
    const uint64_t w = P.rstate[rows[j]];
    const uint32_t c = round_start_count(w, round);
    if (c < bc) {
      bc = c;
      best = rows[j];
      bw = w;
    }
  }
  const uint32_t slot = round_add(&P.rstate[best], bw, round, P.ctl);
  if (slot < P.W) {
    P.pm_key[(uint64_t)best * P.W + slot] = key;
    P.pm_pair[(uint64_t)best * P.W + slot] = P.pair[i];
  } else {
    set_err(P.ctl, kErrOverflow);
  }
}

template <bool MULTI>
__global__ void k_pm_masks(BOLT_PLAN_ARGS) {
  BOLT_PLAN;
  uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= P.R) return;
  const uint32_t cnt = (uint32_t)(P.rstate[r] & kCntMask);
  uint32_t c = cnt < P.W ? cnt : P.W;
  P.pm_mask[r] = c >= 32 ? 0xFFFFFFFFu : ((1u << c) - 1);
}

// Duplicate check: the keys, sorted by the same network, are distinct iff no
// two neighbours are equal.  Padding uses the largest key, so real copies of
// that key are counted apart (bsum[nbs]).
template <bool MULTI>
__global__ void k_dup_fill(BOLT_PLAN_ARGS) {
  BOLT_PLAN;
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P.npad) return;
  const uint64_t k = i < P.n ? P.keys[i] : kNone64;
  P.tag[i] = k;
  if (i < P.n && k == kNone64) atomicAdd(&P.bsum[P.nbs], 1u);
}

template <bool MULTI>
__global__ void k_dup_adjacent(BOLT_PLAN_ARGS) {
  BOLT_PLAN;
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool dup = i + 1 < P.npad && P.tag[i] == P.tag[i + 1] && P.tag[i] != kNone64;
  if (__any(dup) && (threadIdx.x & 63) == 0) set_err(P.ctl, kErrDup);
  if (i == 0 && P.bsum[P.nbs] > 1) set_err(P.ctl, kErrDup);
}

template <bool MULTI>
__global__ void k_build_finish(BOLT_PLAN_ARGS) {
  BOLT_PLAN;
  if (threadIdx.x || blockIdx.x) return;
  P.ctl->live = P.n;
  P.ctl->steps = 0;
}

// Decomposed store: the free-address ring holds the pool entries the HBM
// bins' items left free, in address order (H = items of the HBM bins, the
// scanned load at bin K; K < B, so start[K] exists).
template <bool MULTI>
__global__ void k_ring_init(BOLT_PLAN_ARGS) {
  BOLT_PLAN;
  if (!P.decomp) return;
  const uint64_t H = P.start[P.K];
  const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < P.pool) P.ring[j] = H + j < P.pool ? (uint32_t)(H + j) : kNone;
  if (j == 0) {
    Ctl* c = P.ctl;
    c->ring_head = 0;
    c->ring_tail = H < P.pool ? P.pool - H : 0;
    c->ring_take = 0;
    c->ring_give = 0;
    c->pool_live = H;
    c->hbm_live = H;
    c->stash_live = 0;
    if (H > P.hbm_bound) set_err(c, kErrOverflow);
  }
}

// ---------------------------------------------------------------------------
// Host side: plans, one scratch arena per call, and the launch sequence
// shared by the one-map and the many-map forms.
// ---------------------------------------------------------------------------

static uint32_t blocks_for(uint64_t n, uint32_t nt) { return (uint32_t)((n + nt - 1) / nt); }
static uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

// Scratch bytes of one map's build of n keys.
static uint64_t build_scratch_bytes(const Sizes& s, uint64_t n) {
  uint64_t npad = 1;
  while (npad < n) npad <<= 1;
  const uint64_t nn = n ? n : 1;
  const uint64_t nbs = (s.B + kScanChunk - 1) / kScanChunk;
  return align256(nn * 8) + align256(nn * 4) + align256(npad * 8) + 2 * align256(s.BZ * 8) + align256(s.B * 4) +
         align256((nbs + 1) * 4) + align256(s.R * 8);
}

// Fills one map's plan; carves its scratch from `arena` (advanced).
static void plan_build(bolt_map* m, const uint64_t* keys, const void* vals, uint64_t n, uint8_t*& arena,
                       BuildPlan& P) {
  const Sizes& s = m->s;
  memset(&P, 0, sizeof(P));
  uint64_t npad = 1;
  while (npad < n) npad <<= 1;
  const uint64_t nn = n ? n : 1;
  P.ctl = m->ctl;
  P.keys = keys;
  P.vals = reinterpret_cast<const uint64_t*>(vals);
  P.n = n;
  P.npad = npad;
  P.B = s.B;
  P.K = s.K;
  P.BZ = s.BZ;
  P.R = s.R;
  P.pw = s.page_bytes / 8;
  P.rs = (s.B + 15) / 16;
  P.rsm = (s.R + 15) / 16;
  P.Z = (uint32_t)s.Z;
  P.vw = s.vs / 8;
  P.W = (uint32_t)s.W;
  P.d = (uint32_t)s.d;
  P.nbs = (uint32_t)((s.B + kScanChunk - 1) / kScanChunk);
  P.hbm = reinterpret_cast<uint64_t*>(m->hbm);
  P.obs = reinterpret_cast<uint64_t*>(m->obs);
  P.tags = reinterpret_cast<uint64_t*>(m->tags);
  P.pver = m->pver;
  P.load = m->load;
  P.load0 = m->load0;
  P.pm_key = m->pm_key;
  P.pm_pair = m->pm_pair;
  P.pm_mask = m->pm_mask;
  P.decomp = (m->p.flags & BOLT_F_DECOMPOSED) ? 1 : 0;
  P.pool = s.P;
  P.hbm_bound = s.hbm_bound;
  P.ring = m->ring;
  P.st_key = m->st_key;
  P.st_val = reinterpret_cast<uint64_t*>(m->st_val);
  P.st_dest = m->st_dest;
  P.st_dead = m->st_dead;
  P.rev_cnt = m->rev_cnt;
  P.rev_idx = m->rev_idx;
  auto take = [&arena](uint64_t bytes) {
    uint8_t* p = arena;
    arena += align256(bytes);
    return p;
  };
  P.pair = reinterpret_cast<uint2*>(take(nn * 8));
  P.dest = reinterpret_cast<uint32_t*>(take(nn * 4));
  P.tag = reinterpret_cast<uint64_t*>(take(npad * 8));
  P.elem = reinterpret_cast<uint64_t*>(take(s.BZ * 8));
  P.tmp = reinterpret_cast<uint64_t*>(take(s.BZ * 8));
  P.start = reinterpret_cast<uint32_t*>(take(s.B * 4));
  P.bsum = reinterpret_cast<uint32_t*>(take(((uint64_t)P.nbs + 1) * 4));
  P.rstate = reinterpret_cast<uint64_t*>(take(s.R * 8));
  P.tlog = nullptr;
  if (m->tlog) {
    if (m->tlog_used + s.M <= m->tlog_cap) {
      P.tlog = m->tlog + m->tlog_used;
      TraceSeg g{0, m->tlog_used, 0, s.M};
      m->segs.push_back(g);
      m->tlog_used += s.M;
    } else {
      m->tlog_lost = true;
    }
  }
}

#define BL(K, gx, nt, ...) hipLaunchKernelGGL(K<MULTI>, dim3((gx), C), dim3(nt), 0, st, p1, tab, ##__VA_ARGS__)
#define BLS(K, gx, nt, ...) hipLaunchKernelGGL(K<MULTI>, dim3((gx), C), dim3(nt), 0, side, p1, tab, ##__VA_ARGS__)

// The build sequence (a1 .. a7 and the duplicate check).  The grids and
// trip counts come from the largest map; each map's blocks past its own
// sizes return at once.
template <bool MULTI>
static void build_launches(const std::vector<BuildPlan>& plans, const BuildPlan* tab, const NetSeg* dsort,
                           const NetSeg* dexp, hipStream_t st, hipStream_t side, hipEvent_t ev_fork,
                           hipEvent_t ev_join, KernelTimer* tm) {
  const BuildPlan& p1 = plans[0];
  const uint32_t C = MULTI ? (uint32_t)plans.size() : 1;
  uint64_t n = 0, npad = 0, B = 0, BZ = 0, R = 0, nbs = 0, rp = 0, rm = 0;
  for (const BuildPlan& P : plans) {
    n = std::max(n, P.n);
    npad = std::max(npad, P.npad);
    B = std::max(B, P.B);
    BZ = std::max(BZ, P.BZ);
    R = std::max(R, P.R);
    nbs = std::max(nbs, (uint64_t)P.nbs);
    rp = std::max(rp, (P.n + P.rs - 1) / P.rs);
    rm = std::max(rm, (P.n + P.rsm - 1) / P.rsm);
  }
  uint64_t rs_max = 0, rsm_max = 0;
  for (const BuildPlan& P : plans) {
    rs_max = std::max(rs_max, std::min(P.rs, P.n));
    rsm_max = std::max(rsm_max, std::min(P.rsm, P.n));
  }
  const uint32_t NT = 256;
  {
    TimedScope ts(tm, kkBuildMisc, st);
    BL(k_build_zero, blocks_for(std::max(B, R), NT), NT);
  }
  // a1
  if (n) {
    TimedScope ts(tm, kkPairs, st);
    BL(k_build_pairs, blocks_for(n, NT), NT);
  }
  // a7 on the side stream: the position-map rounds need only the keys and
  // their pairs, so their chain of small launches overlaps a2 .. a6
  (void)hipEventRecord(ev_fork, st);
  (void)hipStreamWaitEvent(side, ev_fork, 0);
  for (uint32_t r = 1; r <= rm; ++r) {
    TimedScope ts(tm, kkPmBuild, side);
    BLS(k_pm_round, blocks_for(rsm_max, NT), NT, r);
  }
  {
    TimedScope ts(tm, kkPmBuild, side);
    BLS(k_pm_masks, blocks_for(R, NT), NT);
  }
  (void)hipEventRecord(ev_join, side);
  // a2: rounds of ceil(B/16) keys
  for (uint32_t r = 1; r <= rp; ++r) {
    {
      TimedScope ts(tm, kkP2C, st);
      BL(k_p2c_decide, blocks_for(rs_max, NT), NT, r);
    }
    TimedScope ts(tm, kkP2C, st);
    BL(k_p2c_add, blocks_for(rs_max, NT), NT, r);
  }
  {
    TimedScope ts(tm, kkBuildMisc, st);
    BL(k_check_loads, blocks_for(B, NT), NT);
  }
  // a3
  {
    TimedScope ts(tm, kkBuildMisc, st);
    BL(k_make_tags, blocks_for(npad, NT), NT);
  }
  if (MULTI)
    launch_bitonic_sort_many(dsort, C, npad, st);
  else
    launch_bitonic_sort(p1.tag, p1.npad, st, tm);
  // a4
  {
    TimedScope ts(tm, kkScan, st);
    BL(k_scan_reduce, (uint32_t)nbs, kScanNT);
    BL(k_scan_top, 1, kScanNT);
    BL(k_scan_down, (uint32_t)nbs, kScanNT);
  }
  {
    TimedScope ts(tm, kkScan, st);
    BL(k_make_elems, blocks_for(BZ, NT), NT);
  }
  // a5
  uint32_t flip = 0;
  if (MULTI)
    flip = launch_expand_many(dexp, C, BZ, st) ? 1 : 0;
  else
    flip = launch_expand_inplace(p1.elem, p1.tmp, p1.BZ, st, tm) != p1.elem ? 1 : 0;
  // a6
  {
    uint64_t lds = 0;  // sealed maps: four pages per workgroup in LDS
    for (const BuildPlan& P : plans)
      if (P.tags) lds = std::max(lds, 4 * P.pw * 8);
    TimedScope ts(tm, kkWriteout, st);
    hipLaunchKernelGGL(k_writeout<MULTI>, dim3(blocks_for(B, 4), C), dim3(256), lds, st, p1, tab, flip);
  }
  {
    uint64_t pool = 0;  // decomposed stores only
    for (const BuildPlan& P : plans)
      if (P.decomp) pool = std::max(pool, P.pool);
    if (pool) {
      TimedScope ts(tm, kkBuildMisc, st);
      BL(k_ring_init, blocks_for(pool, NT), NT);
    }
  }
  // duplicate keys (the tag buffer is free after the write-out)
  if (n) {
    {
      TimedScope ts(tm, kkDupcheck, st);
      BL(k_dup_fill, blocks_for(npad, NT), NT);
    }
    if (MULTI)
      launch_bitonic_sort_many(dsort, C, npad, st);
    else
      launch_bitonic_sort(p1.tag, p1.npad, st, tm);
    TimedScope ts(tm, kkDupcheck, st);
    BL(k_dup_adjacent, blocks_for(npad, NT), NT);
  }
  (void)hipStreamWaitEvent(st, ev_join, 0);
  {
    TimedScope ts(tm, kkBuildMisc, st);
    BL(k_build_finish, 1, 64);
  }
}

#undef BL
#undef BLS

int run_build(bolt_map* m, const uint64_t* keys, const void* vals, uint64_t n, hipStream_t st) {
  uint8_t* arena = nullptr;
  if (hipMallocAsync((void**)&arena, build_scratch_bytes(m->s, n), st) != hipSuccess) return BOLT_ENOMEM;
  std::vector<BuildPlan> plans(1);
  uint8_t* cur = arena;
  plan_build(m, keys, vals, n, cur, plans[0]);
  build_launches<false>(plans, nullptr, nullptr, nullptr, st, m->side, m->ev_fork, m->ev_join, m->timer);
  (void)hipFreeAsync(arena, st);
  return hipGetLastError() == hipSuccess ? BOLT_OK : BOLT_EHIP;
}

int run_build_many(bolt_map* const* maps, const uint64_t* const* keys, const void* const* vals, const uint64_t* n,
                   uint32_t count, hipStream_t st) {
  uint64_t bytes = align256((uint64_t)count * sizeof(BuildPlan)) + 2 * align256((uint64_t)count * sizeof(NetSeg));
  for (uint32_t i = 0; i < count; ++i) bytes += build_scratch_bytes(maps[i]->s, n[i]);
  uint8_t* arena = nullptr;
  if (hipMallocAsync((void**)&arena, bytes, st) != hipSuccess) return BOLT_ENOMEM;
  BuildPlan* dtab = reinterpret_cast<BuildPlan*>(arena);
  NetSeg* dsort = reinterpret_cast<NetSeg*>(arena + align256((uint64_t)count * sizeof(BuildPlan)));
  NetSeg* dexp = dsort + count;  // same 256-byte alignment not needed for the second table
  uint8_t* cur = arena + align256((uint64_t)count * sizeof(BuildPlan)) + 2 * align256((uint64_t)count * sizeof(NetSeg));
  std::vector<BuildPlan> plans(count);
  std::vector<NetSeg> segs(2 * (size_t)count);
  for (uint32_t i = 0; i < count; ++i) {
    plan_build(maps[i], keys[i], vals[i], n[i], cur, plans[i]);
    segs[i] = NetSeg{plans[i].tag, nullptr, plans[i].npad};
    segs[count + i] = NetSeg{plans[i].elem, plans[i].tmp, plans[i].BZ};
  }
  hipError_t e = hipMemcpyAsync(dtab, plans.data(), count * sizeof(BuildPlan), hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dsort, segs.data(), 2 * (size_t)count * sizeof(NetSeg), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) {
    (void)hipFreeAsync(arena, st);
    return BOLT_EHIP;
  }
  build_launches<true>(plans, dtab, dsort, dexp, st, maps[0]->side, maps[0]->ev_fork, maps[0]->ev_join, nullptr);
  (void)hipFreeAsync(arena, st);
  return hipGetLastError() == hipSuccess ? BOLT_OK : BOLT_EHIP;
}

}  // namespace bolt
