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
#include <algorithm>

#include "bolt_impl.h"

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

__global__ __launch_bounds__(kScanNT) void k_scan_reduce(const uint32_t* __restrict__ in, uint64_t n,
                                                         uint32_t* __restrict__ bsum) {
  const uint64_t base = (uint64_t)blockIdx.x * kScanChunk + (uint64_t)threadIdx.x * kScanPer;
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) s += base + i < n ? in[base + i] : 0;
  __shared__ uint32_t tot;
  block_excl_scan<kScanNT>(s, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// Exclusive scan of nb block sums in one block, chunk by chunk.
__global__ __launch_bounds__(kScanNT) void k_scan_top(uint32_t* bsum, uint32_t nb) {
  __shared__ uint32_t tot;
  uint32_t carry = 0;
  for (uint32_t c = 0; c < nb; c += kScanNT) {
    uint32_t i = c + threadIdx.x;
    uint32_t v = i < nb ? bsum[i] : 0;
    uint32_t e = block_excl_scan<kScanNT>(v, &tot);
    __syncthreads();
    if (i < nb) bsum[i] = carry + e;
    carry += tot;
    __syncthreads();
  }
}

__global__ __launch_bounds__(kScanNT) void k_scan_down(const uint32_t* __restrict__ in, uint64_t n,
                                                       const uint32_t* __restrict__ bsum, uint32_t* __restrict__ out) {
  const uint64_t base = (uint64_t)blockIdx.x * kScanChunk + (uint64_t)threadIdx.x * kScanPer;
  uint32_t v[kScanPer];
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    v[i] = base + i < n ? in[base + i] : 0;
    s += v[i];
  }
  __shared__ uint32_t tot;
  uint32_t e = block_excl_scan<kScanNT>(s, &tot) + bsum[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    if (base + i < n) out[base + i] = e;
    e += v[i];
  }
}

static void launch_excl_scan(const uint32_t* in, uint64_t n, uint32_t* bsum, uint32_t* out, hipStream_t st) {
  uint32_t nb = (uint32_t)((n + kScanChunk - 1) / kScanChunk);
  hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kScanNT), 0, st, in, n, bsum);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanNT), 0, st, bsum, nb);
  hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(kScanNT), 0, st, in, n, bsum, out);
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

__global__ void k_build_pairs(const Ctl* ctl, const uint64_t* __restrict__ keys, uint64_t n, uint64_t B,
                              uint2* __restrict__ pair) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t hk[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) hk[j] = ctl->hkey[j];
  uint64_t w[4];
  prf4(hk, kDomPair, keys[i], w);
  uint32_t a, b;
  pair_of(w[0], w[1], B, a, b);
  pair[i] = make_uint2(a, b);
}

__global__ void k_p2c_decide(const uint2* __restrict__ pair, const uint32_t* __restrict__ load, uint64_t r0,
                             uint64_t r1, uint32_t* __restrict__ dest) {
  uint64_t i = r0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= r1) return;
  uint2 p = pair[i];
  dest[i] = load[p.y] < load[p.x] ? p.y : p.x;
}

__global__ void k_p2c_add(const uint32_t* __restrict__ dest, uint64_t r0, uint64_t r1, uint32_t* load) {
  uint64_t i = r0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= r1) return;
  atomicAdd(&load[dest[i]], 1u);
}

__global__ void k_check_loads(const uint32_t* __restrict__ load, uint64_t B, uint32_t Z, Ctl* ctl) {
  uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool bad = b < B && load[b] > Z;
  if (__any(bad) && (threadIdx.x & 63) == 0) set_err(ctl, kErrOverflow);
}

// ---------------------------------------------------------------------------
// a3 + a4
// ---------------------------------------------------------------------------

__global__ void k_make_tags(const uint32_t* __restrict__ dest, uint64_t n, uint64_t npad, uint64_t* __restrict__ tag) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npad) return;
  uint64_t b = i < n ? dest[i] : 0xFFFFFFFFull;
  tag[i] = (b << 32) | (uint32_t)i;
}

// Element for slot placement: (bin * Z + rank) << 32 | input index.
__global__ void k_make_elems(const uint64_t* __restrict__ tag, uint64_t n, const uint32_t* __restrict__ start,
                             uint64_t B, uint32_t Z, uint64_t BZ, uint64_t* __restrict__ elem, Ctl* ctl) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= BZ) return;
  uint64_t e = kNone64;
  if (i < n) {
    uint64_t t = tag[i];
    uint32_t b = (uint32_t)(t >> 32);
    uint64_t rank = b < B ? i - start[b] : Z;
    if (rank < Z)
      e = (((uint64_t)b * Z + rank) << 32) | (uint32_t)t;
    else
      set_err(ctl, kErrOverflow);
  }
  elem[i] = e;
}

// ---------------------------------------------------------------------------
// a6: one wave per bin.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_writeout(const uint64_t* __restrict__ elem, const uint64_t* __restrict__ keys,
                                                  const uint64_t* __restrict__ vals, uint64_t B, uint64_t K, uint32_t Z,
                                                  uint32_t vw, uint64_t pw, uint64_t* __restrict__ hbm,
                                                  uint64_t* __restrict__ obs, uint32_t* __restrict__ tlog) {
  __shared__ uint32_t by_rank[4][64];
  __shared__ uint64_t key_rank[4][64];
  const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint64_t b = (uint64_t)blockIdx.x * 4 + wid;
  const bool active = b < B;  // no early return: the barrier below needs every wave
  uint32_t src = kNone;
  uint64_t key = 0;
  if (active && lane < Z) {
    uint64_t e = elem[b * Z + lane];
    if (e != kNone64) {
      src = (uint32_t)e;
      key = keys[src];
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
  if (!active) return;
  uint64_t* dst = b < K ? hbm + b * pw : obs + (b - K) * pw;
  for (uint64_t w = lane; w < pw; w += 64) {
    uint64_t v = 0;
    if (w == 0) {
      v = cnt >= 64 ? kNone64 : ((1ull << cnt) - 1);
    } else if (w <= Z) {
      uint32_t j = (uint32_t)w - 1;
      v = j < cnt ? key_rank[wid][j] : 0;
    } else if (w < 1 + Z + (uint64_t)Z * vw) {
      uint64_t off = w - 1 - Z;
      uint32_t j = (uint32_t)(off / vw), o = (uint32_t)(off % vw);
      v = j < cnt ? vals[(uint64_t)by_rank[wid][j] * vw + o] : 0;
    }
    dst[w] = v;
  }
  if (tlog && b >= K && lane == 0) tlog[b - K] = (uint32_t)(b - K);
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

__global__ void k_pm_decide(const Ctl* ctl, const uint64_t* __restrict__ keys, uint64_t r0, uint64_t r1, uint64_t R,
                            uint32_t d, const uint32_t* __restrict__ rowcnt, uint32_t* __restrict__ rowsel) {
  uint64_t i = r0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= r1) return;
  uint32_t hk[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) hk[j] = ctl->hkey[j];
  uint32_t rows[4];
  pm_rows_of(hk, keys[i], R, d, rows);
  uint32_t best = rows[0], bc = rowcnt[rows[0]];
  for (uint32_t j = 1; j < d; ++j) {
    uint32_t c = rowcnt[rows[j]];
    if (c < bc) {
      bc = c;
      best = rows[j];
    }
  }
  rowsel[i] = best;
}

__global__ void k_pm_add(const uint64_t* __restrict__ keys, const uint2* __restrict__ pair,
                         const uint32_t* __restrict__ rowsel, uint64_t r0, uint64_t r1, uint32_t W, uint32_t* rowcnt,
                         uint64_t* __restrict__ pm_key, uint2* __restrict__ pm_pair, Ctl* ctl) {
  uint64_t i = r0 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= r1) return;
  uint32_t r = rowsel[i];
  uint32_t slot = atomicAdd(&rowcnt[r], 1u);
  if (slot < W) {
    pm_key[(uint64_t)r * W + slot] = keys[i];
    pm_pair[(uint64_t)r * W + slot] = pair[i];
  } else {
    set_err(ctl, kErrOverflow);
  }
}

__global__ void k_pm_masks(const uint32_t* __restrict__ rowcnt, uint64_t R, uint32_t W, uint32_t* __restrict__ mask) {
  uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  uint32_t c = rowcnt[r] < W ? rowcnt[r] : W;
  mask[r] = c >= 32 ? 0xFFFFFFFFu : ((1u << c) - 1);
}

// Duplicate check: the keys, sorted by the same network, are distinct iff no
// two neighbours are equal.  Padding uses the largest key, so real copies of
// that key are counted apart.
__global__ void k_dup_fill(const uint64_t* __restrict__ keys, uint64_t n, uint64_t npad, uint64_t* __restrict__ tag,
                           uint32_t* n_max) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npad) return;
  const uint64_t k = i < n ? keys[i] : kNone64;
  tag[i] = k;
  if (i < n && k == kNone64) atomicAdd(n_max, 1u);
}

__global__ void k_dup_adjacent(const uint64_t* __restrict__ tag, uint64_t npad, const uint32_t* n_max, Ctl* ctl) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool dup = i + 1 < npad && tag[i] == tag[i + 1] && tag[i] != kNone64;
  if (__any(dup) && (threadIdx.x & 63) == 0) set_err(ctl, kErrDup);
  if (i == 0 && *n_max > 1) set_err(ctl, kErrDup);
}

__global__ void k_build_finish(Ctl* ctl, uint64_t n) {
  if (threadIdx.x || blockIdx.x) return;
  ctl->live = n;
  ctl->steps = 0;
}

// ---------------------------------------------------------------------------

static uint32_t blocks_for(uint64_t n, uint32_t nt) { return (uint32_t)((n + nt - 1) / nt); }

static void free_build_scratch(BuildScratch& b, hipStream_t st) {
  void* ptrs[] = {b.pair, b.dest, b.tag, b.elem, b.tmp, b.start, b.bsum, b.rowsel, b.rowcnt};
  for (void* p : ptrs)
    if (p) (void)hipFreeAsync(p, st);
}

int run_build(bolt_map* m, const uint64_t* keys, const void* vals, uint64_t n, hipStream_t st) {
  const Sizes& s = m->s;
  uint64_t npad = 1;
  while (npad < n) npad <<= 1;
  BuildScratch b{};
  size_t nn = n ? n : 1;
  uint32_t nbs = (uint32_t)((s.B + kScanChunk - 1) / kScanChunk);
  hipError_t e = hipSuccess;
  e = e ? e : hipMallocAsync((void**)&b.pair, nn * sizeof(uint2), st);
  e = e ? e : hipMallocAsync((void**)&b.dest, nn * sizeof(uint32_t), st);
  e = e ? e : hipMallocAsync((void**)&b.tag, npad * sizeof(uint64_t), st);
  e = e ? e : hipMallocAsync((void**)&b.elem, s.BZ * sizeof(uint64_t), st);
  e = e ? e : hipMallocAsync((void**)&b.tmp, s.BZ * sizeof(uint64_t), st);
  e = e ? e : hipMallocAsync((void**)&b.start, s.B * sizeof(uint32_t), st);
  e = e ? e : hipMallocAsync((void**)&b.bsum, (nbs + 1) * sizeof(uint32_t), st);
  e = e ? e : hipMallocAsync((void**)&b.rowsel, nn * sizeof(uint32_t), st);
  e = e ? e : hipMallocAsync((void**)&b.rowcnt, s.R * sizeof(uint32_t), st);
  if (e != hipSuccess) {
    free_build_scratch(b, st);
    return BOLT_ENOMEM;
  }
  const uint32_t NT = 256;
  // a1
  if (n) {
    TimedScope ts(m->timer, kkPairs, st);
    hipLaunchKernelGGL(k_build_pairs, dim3(blocks_for(n, NT)), dim3(NT), 0, st, m->ctl, keys, n, s.B, b.pair);
  }
  // a2
  const uint64_t rs = (s.B + 15) / 16;
  {
    for (uint64_t r0 = 0; r0 < n; r0 += rs) {
      uint64_t r1 = r0 + rs < n ? r0 + rs : n;
      {
        TimedScope ts(m->timer, kkP2C, st);
        hipLaunchKernelGGL(k_p2c_decide, dim3(blocks_for(r1 - r0, NT)), dim3(NT), 0, st, b.pair, m->load, r0, r1,
                           b.dest);
      }
      {
        TimedScope ts(m->timer, kkP2C, st);
        hipLaunchKernelGGL(k_p2c_add, dim3(blocks_for(r1 - r0, NT)), dim3(NT), 0, st, b.dest, r0, r1, m->load);
      }
    }
  }
  {
    TimedScope ts(m->timer, kkBuildMisc, st);
    hipLaunchKernelGGL(k_check_loads, dim3(blocks_for(s.B, NT)), dim3(NT), 0, st, m->load, s.B, (uint32_t)s.Z, m->ctl);
  }
  // a3
  {
    TimedScope ts(m->timer, kkBuildMisc, st);
    hipLaunchKernelGGL(k_make_tags, dim3(blocks_for(npad, NT)), dim3(NT), 0, st, b.dest, n, npad, b.tag);
  }
  launch_bitonic_sort(b.tag, npad, st, m->timer);
  // a4
  {
    TimedScope ts(m->timer, kkScan, st);
    launch_excl_scan(m->load, s.B, b.bsum, b.start, st);
  }
  {
    TimedScope ts(m->timer, kkScan, st);
    hipLaunchKernelGGL(k_make_elems, dim3(blocks_for(s.BZ, NT)), dim3(NT), 0, st, b.tag, n, b.start, s.B, (uint32_t)s.Z,
                       s.BZ, b.elem, m->ctl);
  }
  // a5
  launch_expand(b.elem, b.tmp, s.BZ, st, m->timer);
  // a6
  uint32_t* tl = nullptr;
  if (m->tlog) {
    if (m->tlog_used + s.M <= m->tlog_cap) {
      tl = m->tlog + m->tlog_used;
      TraceSeg g{0, m->tlog_used, 0, s.M};
      m->segs.push_back(g);
      m->tlog_used += s.M;
    } else {
      m->tlog_lost = true;
    }
  }
  {
    TimedScope ts(m->timer, kkWriteout, st);
    hipLaunchKernelGGL(k_writeout, dim3(blocks_for(s.B, 4)), dim3(256), 0, st, b.elem, keys,
                       reinterpret_cast<const uint64_t*>(vals), s.B, s.K, (uint32_t)s.Z, s.vs / 8, s.page_bytes / 8,
                       reinterpret_cast<uint64_t*>(m->hbm), reinterpret_cast<uint64_t*>(m->obs), tl);
  }
  // a7
  (void)hipMemsetAsync(b.rowcnt, 0, s.R * sizeof(uint32_t), st);
  const uint64_t rsm = (s.R + 15) / 16;
  {
    for (uint64_t r0 = 0; r0 < n; r0 += rsm) {
      uint64_t r1 = r0 + rsm < n ? r0 + rsm : n;
      {
        TimedScope ts(m->timer, kkPmBuild, st);
        hipLaunchKernelGGL(k_pm_decide, dim3(blocks_for(r1 - r0, NT)), dim3(NT), 0, st, m->ctl, keys, r0, r1, s.R,
                           (uint32_t)s.d, b.rowcnt, b.rowsel);
      }
      {
        TimedScope ts(m->timer, kkPmBuild, st);
        hipLaunchKernelGGL(k_pm_add, dim3(blocks_for(r1 - r0, NT)), dim3(NT), 0, st, keys, b.pair, b.rowsel, r0, r1,
                           (uint32_t)s.W, b.rowcnt, m->pm_key, m->pm_pair, m->ctl);
      }
    }
  }
  {
    TimedScope ts(m->timer, kkPmBuild, st);
    hipLaunchKernelGGL(k_pm_masks, dim3(blocks_for(s.R, NT)), dim3(NT), 0, st, b.rowcnt, s.R, (uint32_t)s.W, m->pm_mask);
  }
  // duplicate keys (the tag buffer is free after the write-out)
  if (n) {
    (void)hipMemsetAsync(b.bsum + nbs, 0, sizeof(uint32_t), st);
    {
      TimedScope ts(m->timer, kkDupcheck, st);
      hipLaunchKernelGGL(k_dup_fill, dim3(blocks_for(npad, NT)), dim3(NT), 0, st, keys, n, npad, b.tag, b.bsum + nbs);
    }
    launch_bitonic_sort(b.tag, npad, st, m->timer);
    TimedScope ts(m->timer, kkDupcheck, st);
    hipLaunchKernelGGL(k_dup_adjacent, dim3(blocks_for(npad, NT)), dim3(NT), 0, st, b.tag, npad, b.bsum + nbs, m->ctl);
  }
  {
    TimedScope ts(m->timer, kkBuildMisc, st);
    hipLaunchKernelGGL(k_build_finish, dim3(1), dim3(64), 0, st, m->ctl, n);
  }
  free_build_scratch(b, st);
  return hipGetLastError() == hipSuccess ? BOLT_OK : BOLT_EHIP;
}

}  // namespace bolt
