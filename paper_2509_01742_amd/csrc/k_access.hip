// Batched oblivious access (Alg. 1 per command, in the module order of
// Sec. 5.1): decode, key search, value access, remap + eviction, response.
//
// One batch of q commands runs as six kernels on one stream:
//   dedup     sort (key, index) in LDS; leader = first command of each key;
//             for every command the last PUT/DEL of its key before it
//   fetch     one wave per command: tape T(s) -> fetch pair F(s) and remap
//             pair R(s); leaders look their key up in the position map (d
//             rows); read both bins whole (observable pages are copied to
//             a staging area); the leader of a mapped key finds and removes
//             its item (page slot or stash entry); elect one writer per bin
//   resolve   responses of every command in index order (sequential
//             semantics of the batch)
//   remap     one workgroup: keys present at the end get R(s) and P2C over
//             the post-removal loads, in rounds of ceil(B/16); the item goes
//             to the stash pool listed under its bin; position-map updates,
//             deletes, then inserts in rounds of ceil(R/16)
//   writeback one wave per candidate bin: the elected writer rebuilds the
//             bin as survivors + every live stash item listed for it,
//             canonical order, and writes it whole (observable pages once
//             each)
//   finish    counters, stash bound
#include "bolt_impl.h"

namespace bolt {

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
  // exclusive within the wave
  uint32_t wex = __shfl_up(inc, 1, 64);
  if (lane == 0) wex = 0;
  uint32_t r = MAX ? (before > wex ? before : wex) : before + wex;
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------------------
// dedup + fold structure (one workgroup)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kDedupNT) void k_acc_dedup(const uint8_t* __restrict__ ops,
                                                        const uint64_t* __restrict__ keys, uint32_t q, Ctl* ctl,
                                                        uint32_t* __restrict__ leader, uint32_t* __restrict__ prevw,
                                                        uint32_t* __restrict__ lastw) {
  __shared__ uint64_t skey[kMaxBatch];
  __shared__ uint32_t sidx[kMaxBatch];
  __shared__ uint32_t tot;
  __shared__ uint32_t bad;
  if (threadIdx.x == 0) bad = 0;
  uint32_t npad = 1;
  while (npad < q) npad <<= 1;
  __syncthreads();
  for (uint32_t r = threadIdx.x; r < npad; r += kDedupNT) {
    bool real = r < q;
    skey[r] = real ? keys[r] : kNone64;
    sidx[r] = real ? r : kNone;
    if (real && ops[r] > 2) bad = 1;
  }
  __syncthreads();
  if (threadIdx.x == 0) ctl->reject = bad;
  if (bad) return;  // the whole block sees the same value
  // bitonic sort by (key, index), ascending
  for (uint32_t k = 2; k <= npad; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t p = threadIdx.x; p < npad / 2; p += kDedupNT) {
        uint32_t i = ((p & ~(j - 1)) << 1) | (p & (j - 1));
        uint32_t l = i + j;
        bool asc = (i & k) == 0;
        uint64_t ka = skey[i], kb = skey[l];
        uint32_t ia = sidx[i], ib = sidx[l];
        bool gt = ka > kb || (ka == kb && ia > ib);
        if (gt == asc) {
          skey[i] = kb;
          skey[l] = ka;
          sidx[i] = ib;
          sidx[l] = ia;
        }
      }
      __syncthreads();
    }
  }
  // Each thread owns kDedupPer consecutive sorted positions.  Values are
  // stored +1 so that 0 means "none".
  const uint32_t r0 = threadIdx.x * kDedupPer;
  uint32_t rs[kDedupPer], wp[kDedupPer];
  uint32_t run = 0, wmax = 0;
  for (uint32_t t = 0; t < kDedupPer; ++t) {
    uint32_t r = r0 + t;
    if (r < q) {
      bool head = r == 0 || skey[r] != skey[r - 1];
      if (head) run = r + 1;
      rs[t] = run;
      wp[t] = wmax;  // writers strictly before r within this chunk
      if (ops[sidx[r]] != 0) wmax = r + 1;
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
    uint32_t me = sidx[r];
    leader[me] = sidx[start - 1];
    prevw[me] = (w != 0 && w >= start) ? sidx[w - 1] : kNone;
    bool tail = r + 1 == q || skey[r + 1] != skey[r];
    if (tail) {
      uint32_t wl = w;
      if (ops[me] != 0) wl = r + 1;
      lastw[sidx[start - 1]] = (wl != 0 && wl >= start) ? sidx[wl - 1] : kNone;
    }
  }
}

// ---------------------------------------------------------------------------
// fetch: one wave per command
// ---------------------------------------------------------------------------

struct FetchArgs {
  const Ctl* ctl;
  const uint8_t* ops;
  const uint64_t* keys;
  const uint32_t* leader;
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
};

__global__ __launch_bounds__(256) void k_acc_fetch(FetchArgs a) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= a.q) return;
  if (a.ctl->reject || a.ctl->err) return;
  uint32_t hk[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) hk[j] = a.ctl->hkey[j];
  const uint64_t s = a.ctl->steps + i;
  uint64_t w[4];
  prf4(hk, kDomTape, s, w);
  uint32_t f1, f2, r1, r2;
  pair_of(w[0], w[1], a.B, f1, f2);
  pair_of(w[2], w[3], a.B, r1, r2);
  if (lane == 0) a.rpair[i] = make_uint2(r1, r2);
  const uint64_t key = a.keys[i];
  const bool is_leader = a.leader[i] == i;
  // key search (Sec. 5.1 step 3): d rows, 16 lanes per row, 2 slots per lane
  bool hit = false;
  uint32_t hrow = 0, hslot = 0, p1 = f1, p2 = f2;
  if (is_leader) {
    uint32_t rows[4];
    uint64_t g[4];
    prf4(hk, kDomRows, key, g);
#pragma unroll
    for (int j = 0; j < 4; ++j) rows[j] = (uint32_t)__umul64hi(g[j], a.R);
    const uint32_t j = lane >> 4;
    const uint32_t row = rows[j];
    const uint32_t s0 = (lane & 15) * 2;
    bool m0 = false, m1 = false;
    if (j < a.d) {
      const uint32_t mk = a.pm_mask[row];
      if (s0 < a.W && ((mk >> s0) & 1)) m0 = a.pm_key[(uint64_t)row * a.W + s0] == key;
      if (s0 + 1 < a.W && ((mk >> (s0 + 1)) & 1)) m1 = a.pm_key[(uint64_t)row * a.W + s0 + 1] == key;
    }
    const uint64_t bal = __ballot(m0 || m1);
    if (bal) {
      const uint32_t src = __builtin_ctzll(bal);
      const uint32_t slot = s0 + (m0 ? 0 : 1);
      hrow = __shfl(row, src, 64);
      hslot = __shfl(slot, src, 64);
      hit = true;
      const uint2 pp = a.pm_pair[(uint64_t)hrow * a.W + hslot];
      p1 = pp.x;
      p2 = pp.y;
    }
  }
  // value access (Sec. 5.1 step 4): both bins, whole
  bool found = false;
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
    const uint64_t v0 = lane < a.pw ? src[lane] : 0;
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
    for (uint64_t wi = lane + 64; wi < a.pw; wi += 64) {
      const uint64_t v = src[wi];
      if (host) stg[wi] = v;
      if (fslot >= 0 && wi >= vlo && wi < vlo + a.vw) a.fval[(uint64_t)i * a.vw + (wi - vlo)] = v;
    }
    if (fslot >= 0) {
      found = true;
      if (lane == 0) {
        atomicOr((unsigned long long*)&a.rmask[b], (unsigned long long)(1ull << fslot));
        atomicSub(&a.load[b], 1u);
      }
    } else if (search && host) {
      // the stash items listed for this bin
      const uint32_t cnt = a.rev_cnt[b] < 2 * a.Z ? a.rev_cnt[b] : 2 * a.Z;
      int fe = -1;
      for (uint32_t base = 0; base < cnt; base += 64) {
        const uint32_t l = base + lane;
        uint32_t e = kNone;
        bool m = false;
        if (l < cnt) {
          e = a.rev_idx[(uint64_t)b * 2 * a.Z + l];
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
  }
}

// ---------------------------------------------------------------------------
// resolve: responses (one thread per command)
// ---------------------------------------------------------------------------

__global__ void k_acc_resolve(const Ctl* ctl, const uint8_t* __restrict__ ops, const uint64_t* __restrict__ vals_in,
                              const uint32_t* __restrict__ leader, const uint32_t* __restrict__ prevw,
                              const uint32_t* __restrict__ found, const uint64_t* __restrict__ fval, uint32_t q,
                              uint32_t vw, uint64_t* __restrict__ vals_out, uint8_t* __restrict__ status) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= q) return;
  uint64_t* out = vals_out + (uint64_t)i * vw;
  if (ctl->reject || ctl->err) {
    status[i] = 0xFF;
    for (uint32_t o = 0; o < vw; ++o) out[o] = 0;
    return;
  }
  const uint32_t L = leader[i], w = prevw[i];
  const bool present = w != kNone ? ops[w] == 1 : found[L] != 0;
  const uint64_t* src = w != kNone ? vals_in + (uint64_t)w * vw : fval + (uint64_t)L * vw;
  const uint8_t op = ops[i];
  uint8_t st;
  if (op == 0) st = present ? 1 : 0;
  else if (op == 1) st = present ? 1 : 2;
  else st = present ? 3 : 0;
  status[i] = st;
  const bool give = op == 0 && present;
  for (uint32_t o = 0; o < vw; ++o) out[o] = give ? src[o] : 0;
}

// ---------------------------------------------------------------------------
// remap + P2C + position map (one workgroup)
// ---------------------------------------------------------------------------

constexpr uint32_t kRemapNT = 1024;
constexpr uint32_t kRemapPer = kMaxBatch / kRemapNT;

struct RemapArgs {
  Ctl* ctl;
  const uint8_t* ops;
  const uint64_t* keys;
  const uint64_t* vals_in;
  const uint32_t* leader;
  const uint32_t* lastw;
  const uint32_t* hit;
  const uint32_t* hrow;
  const uint32_t* hslot;
  const uint32_t* found;
  const uint64_t* fval;
  const uint2* rpair;
  uint32_t q, epoch, Z, W, d, vw;
  uint64_t B, K, R, P, cap;
  uint32_t* load;
  uint64_t* st_key;
  uint64_t* st_val;
  uint32_t* st_dest;
  uint32_t* st_dead;
  const uint32_t* ring;
  uint32_t* rev_cnt;
  uint32_t* rev_idx;
  uint64_t* claim;
  uint32_t* cand_bin;
  uint64_t* pm_key;
  uint2* pm_pair;
  uint32_t* pm_mask;
};

__global__ __launch_bounds__(kRemapNT) void k_acc_remap(RemapArgs a) {
  __shared__ uint32_t tot;
  __shared__ uint32_t s_skip;
  if (threadIdx.x == 0) s_skip = (a.ctl->reject || a.ctl->err) ? 1 : 0;
  __syncthreads();
  if (s_skip) return;
  const uint32_t i0 = threadIdx.x * kRemapPer;
  // final state of every key in the batch (leaders only)
  uint32_t fin[kRemapPer];  // bit0 present, bit1 hit, bit2 insert
  uint32_t nplace_mine = 0, nins_mine = 0, ndel_mine = 0;
  for (uint32_t t = 0; t < kRemapPer; ++t) {
    const uint32_t i = i0 + t;
    fin[t] = 0;
    if (i >= a.q || a.leader[i] != i) continue;
    const uint32_t lw = a.lastw[i];
    const bool present = lw != kNone ? a.ops[lw] == 1 : a.found[i] != 0;
    const bool h = a.hit[i] != 0;
    fin[t] = (present ? 1u : 0u) | (h ? 2u : 0u);
    nplace_mine += present;
    nins_mine += present && !h;
    ndel_mine += h && !present;
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
  const uint64_t head = a.ctl->ring_head, tail = a.ctl->ring_tail;
  if ((uint64_t)nplace > tail - head) {
    if (threadIdx.x == 0) set_err(a.ctl, kErrOverflow);
    return;  // uniform
  }
  // P2C in rounds of ceil(B/16) over the post-removal loads (Sec. 5.1 step 5)
  const uint64_t rs = (a.B + 15) / 16;
  uint32_t chosen[kRemapPer];
  for (uint64_t r0 = 0; r0 < nplace; r0 += rs) {
    uint32_t o = place0;
    for (uint32_t t = 0; t < kRemapPer; ++t) {
      if (!(fin[t] & 1)) continue;
      if (o >= r0 && o < r0 + rs) {
        const uint2 rp = a.rpair[i0 + t];
        const uint32_t l1 = ld_acq32(&a.load[rp.x]), l2 = ld_acq32(&a.load[rp.y]);
        chosen[t] = l2 < l1 ? rp.y : rp.x;
      }
      ++o;
    }
    __syncthreads();
    o = place0;
    for (uint32_t t = 0; t < kRemapPer; ++t) {
      if (!(fin[t] & 1)) continue;
      if (o >= r0 && o < r0 + rs) {
        const uint32_t old = atomicAdd(&a.load[chosen[t]], 1u);
        if (old + 1 > a.Z) set_err(a.ctl, kErrOverflow);
      }
      ++o;
    }
    __threadfence();
    __syncthreads();
  }
  // place every remapped item in the stash pool, listed under its bin
  uint32_t o = place0;
  for (uint32_t t = 0; t < kRemapPer; ++t) {
    const uint32_t i = i0 + t;
    if (i < a.q) a.cand_bin[2 * a.q + i] = kNone;
    if (!(fin[t] & 1)) continue;
    const uint32_t b = chosen[t];
    const uint32_t e = a.ring[(head + o) % a.P];
    ++o;
    const uint32_t lw = a.lastw[i];
    const uint64_t* src = lw != kNone ? a.vals_in + (uint64_t)lw * a.vw : a.fval + (uint64_t)i * a.vw;
    a.st_key[e] = a.keys[i];
    for (uint32_t x = 0; x < a.vw; ++x) a.st_val[(uint64_t)e * a.vw + x] = src[x];
    a.st_dest[e] = b;
    a.st_dead[e] = 0;
    const uint32_t ls = atomicAdd(&a.rev_cnt[b], 1u);
    if (ls < 2 * a.Z)
      a.rev_idx[(uint64_t)b * 2 * a.Z + ls] = e;
    else
      set_err(a.ctl, kErrOverflow);
    if (b < a.K) {  // HBM bins are rebuilt in this batch
      a.cand_bin[2 * a.q + i] = b;
      atomicMax((unsigned long long*)&a.claim[b], (unsigned long long)claim_tag(a.epoch, 2 * a.q + i));
    }
  }
  // position map: new pairs for keys that stay, deletes ...
  for (uint32_t t = 0; t < kRemapPer; ++t) {
    const uint32_t i = i0 + t;
    if (!(fin[t] & 2)) continue;
    const uint64_t at = (uint64_t)a.hrow[i] * a.W + a.hslot[i];
    if (fin[t] & 1)
      a.pm_pair[at] = a.rpair[i];
    else
      atomicAnd(&a.pm_mask[a.hrow[i]], ~(1u << a.hslot[i]));
  }
  __threadfence();
  __syncthreads();
  // ... then inserts, in rounds of ceil(R/16) that see the row loads at
  // their start; the least loaded of d rows, ties to the lowest choice
  const uint64_t rsm = (a.R + 15) / 16;
  uint32_t rowsel[kRemapPer];
  const uint32_t hk0[8] = {a.ctl->hkey[0], a.ctl->hkey[1], a.ctl->hkey[2], a.ctl->hkey[3],
                           a.ctl->hkey[4], a.ctl->hkey[5], a.ctl->hkey[6], a.ctl->hkey[7]};
  for (uint64_t r0 = 0; r0 < nins; r0 += rsm) {
    uint32_t io = ins0;
    for (uint32_t t = 0; t < kRemapPer; ++t) {
      if ((fin[t] & 3) != 1) continue;
      if (io >= r0 && io < r0 + rsm) {
        uint64_t g[4];
        prf4(hk0, kDomRows, a.keys[i0 + t], g);
        uint32_t best = (uint32_t)__umul64hi(g[0], a.R);
        uint32_t bc = __popc(ld_acq32(&a.pm_mask[best]));
        for (uint32_t j = 1; j < a.d; ++j) {
          const uint32_t r = (uint32_t)__umul64hi(g[j], a.R);
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
        const uint32_t r = rowsel[t];
        const uint32_t full = a.W >= 32 ? 0xFFFFFFFFu : ((1u << a.W) - 1);
        bool done = false;
        for (uint32_t tries = 0; tries < 32 && !done; ++tries) {
          const uint32_t mk = ld_acq32(&a.pm_mask[r]);
          const uint32_t free = ~mk & full;
          if (!free) break;
          const uint32_t bit = free & (0u - free);
          const uint32_t prev = atomicOr(&a.pm_mask[r], bit);
          if (!(prev & bit)) {
            const uint32_t slot = __builtin_ctz(bit);
            a.pm_key[(uint64_t)r * a.W + slot] = a.keys[i0 + t];
            a.pm_pair[(uint64_t)r * a.W + slot] = a.rpair[i0 + t];
            done = true;
          }
        }
        if (!done) set_err(a.ctl, kErrOverflow);
      }
      ++io;
    }
    __threadfence();
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    a.ctl->ring_head = head + nplace;
    a.ctl->n_place = nplace;
    a.ctl->batch_delta = (int64_t)nins - (int64_t)ndel;
    const uint64_t live = a.ctl->live + nins - ndel;
    a.ctl->live = live;
    if (live > a.cap) set_err(a.ctl, kErrFull);
  }
}

// ---------------------------------------------------------------------------
// write-back with eviction: one wave per candidate slot
// ---------------------------------------------------------------------------

struct WbArgs {
  Ctl* ctl;
  uint32_t q, epoch, Z, vw;
  uint64_t K, P, pw;
  const uint32_t* cand_bin;
  const uint64_t* claim;
  uint64_t* rmask;
  uint64_t* stage;
  uint64_t* obs;
  uint64_t* hbm;
  uint32_t* rev_cnt;
  const uint32_t* rev_idx;
  const uint64_t* st_key;
  const uint64_t* st_val;
  uint32_t* st_dead;
  uint32_t* ring;
  uint32_t* tlog_w;  // [3q] or null
};

constexpr uint32_t kWbItems = 192;  // Z survivors + 2Z listed stash entries, Z <= 62

__global__ __launch_bounds__(256) void k_acc_writeback(WbArgs a) {
  __shared__ uint64_t ikey[4][kWbItems];
  __shared__ uint32_t isrc[4][kWbItems];
  __shared__ uint32_t by_rank[4][64];
  const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint32_t s = blockIdx.x * 4 + wid;
  bool active = s < 3 * a.q && !a.ctl->reject && !a.ctl->err;
  uint32_t b = kNone;
  if (active) {
    b = a.cand_bin[s];
    active = b != kNone && a.claim[b] == claim_tag(a.epoch, s);
  }
  const bool host = active && b >= a.K;
  uint64_t* stg = a.stage + (uint64_t)s * a.pw;
  // HBM bins are rebuilt in place: copy the old bin to this slot's stage first
  if (active && !host) {
    for (uint64_t w = lane; w < a.pw; w += 64) stg[w] = a.hbm[(uint64_t)b * a.pw + w];
    __threadfence();
  }
  uint32_t n_items = 0;
  uint32_t n_surv = 0;
  if (active) {
    const uint64_t mask = ld_acq64(&stg[0]);
    const uint64_t rm = a.rmask[b];
    const uint64_t keep = mask & ~rm;
    // survivors, in slot order
    if (lane < a.Z) {
      const bool k = (keep >> lane) & 1;
      const uint64_t kk = ld_acq64(&stg[1 + lane]);
      const uint32_t pos = __popcll(keep & ((1ull << lane) - 1));
      if (k) {
        ikey[wid][pos] = kk;
        isrc[wid][pos] = lane;  // page slot
      }
    }
    n_surv = __popcll(keep);
    // every entry listed under the bin: live ones move in, all are freed
    const uint32_t cnt = a.rev_cnt[b] < 2 * a.Z ? a.rev_cnt[b] : 2 * a.Z;
    uint64_t ring_base = 0;
    if (lane == 0 && cnt) ring_base = atomicAdd((unsigned long long*)&a.ctl->ring_tail, (unsigned long long)cnt);
    ring_base = __shfl(ring_base, 0, 64);
    uint32_t n_alive = 0;
    for (uint32_t base = 0; base < cnt; base += 64) {
      const uint32_t l = base + lane;
      uint32_t e = kNone;
      bool alive = false;
      if (l < cnt) {
        e = a.rev_idx[(uint64_t)b * 2 * a.Z + l];
        alive = !a.st_dead[e];
      }
      const uint64_t bal = __ballot(alive);
      if (alive) {
        const uint32_t pos = n_surv + n_alive + __popcll(bal & ((1ull << lane) - 1));
        if (pos < kWbItems) {
          ikey[wid][pos] = a.st_key[e];
          isrc[wid][pos] = 0x80000000u | e;
        }
      }
      n_alive += __popcll(bal);
      if (l < cnt) {
        a.st_dead[e] = 0;
        a.ring[(ring_base + l) % a.P] = e;
      }
    }
    n_items = n_surv + n_alive;
    if (lane == 0) {
      a.rmask[b] = 0;
      a.rev_cnt[b] = 0;
      if (n_items > a.Z) set_err(a.ctl, kErrOverflow);
    }
  }
  __syncthreads();
  const bool go = active && n_items <= a.Z;  // wave-uniform; every wave reaches both barriers
  // canonical order: ascending key
  if (go && lane < n_items) {
    const uint64_t mine = ikey[wid][lane];
    uint32_t rank = 0;
    for (uint32_t j = 0; j < n_items; ++j) rank += ikey[wid][j] < mine || (ikey[wid][j] == mine && j < lane);
    by_rank[wid][rank] = lane;
  }
  __syncthreads();
  if (!go) return;
  uint64_t* dst = host ? a.obs + (uint64_t)(b - a.K) * a.pw : a.hbm + (uint64_t)b * a.pw;
  for (uint64_t w = lane; w < a.pw; w += 64) {
    uint64_t v = 0;
    if (w == 0) {
      v = n_items >= 64 ? kNone64 : ((1ull << n_items) - 1);
    } else if (w <= a.Z) {
      const uint32_t j = (uint32_t)w - 1;
      v = j < n_items ? ikey[wid][by_rank[wid][j]] : 0;
    } else if (w < 1 + a.Z + (uint64_t)a.Z * a.vw) {
      const uint64_t off = w - 1 - a.Z;
      const uint32_t j = (uint32_t)(off / a.vw), o = (uint32_t)(off % a.vw);
      if (j < n_items) {
        const uint32_t src = isrc[wid][by_rank[wid][j]];
        if (src & 0x80000000u)
          v = a.st_val[(uint64_t)(src & 0x7FFFFFFFu) * a.vw + o];
        else
          v = ld_acq64(&stg[1 + a.Z + (uint64_t)src * a.vw + o]);
      }
    }
    dst[w] = v;
  }
  if (host && lane == 0 && a.tlog_w) a.tlog_w[s] = (uint32_t)(b - a.K);
}

__global__ void k_acc_finish(Ctl* ctl, uint32_t q, uint64_t P, uint64_t stash_bound) {
  if (threadIdx.x || blockIdx.x) return;
  if (ctl->reject) return;
  ctl->steps += q;
  const uint64_t live_stash = P - (ctl->ring_tail - ctl->ring_head);
  if (live_stash > ctl->stash_hw) ctl->stash_hw = live_stash;
  if (live_stash > stash_bound) ctl->err |= kErrOverflow;
}

// Fill of the trace segment of a batch (no memset nodes in captured graphs).
__global__ void k_fill_u32(uint32_t* p, uint64_t n, uint32_t v) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------

int run_access(bolt_map* m, const uint8_t* ops, const uint64_t* keys, const void* vals_in, void* vals_out,
               uint8_t* status, uint32_t q, hipStream_t st) {
  const Sizes& s = m->s;
  const BatchScratch& bs = m->bs;
  const uint32_t epoch = (uint32_t)(m->batches + 1);
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
      hipLaunchKernelGGL(k_fill_u32, dim3((uint32_t)((words + 255) / 256)), dim3(256), 0, st, tlog_r, words, kNone);
    } else {
      m->tlog_lost = true;
    }
  }
  {
    TimedScope ts(m->timer, kkAccDedup, st);
    hipLaunchKernelGGL(k_acc_dedup, dim3(1), dim3(kDedupNT), 0, st, ops, keys, q, m->ctl, bs.leader, bs.prevw, bs.lastw);
  }

  FetchArgs fa;
  fa.ctl = m->ctl;
  fa.ops = ops;
  fa.keys = keys;
  fa.leader = bs.leader;
  fa.q = q;
  fa.epoch = epoch;
  fa.B = s.B;
  fa.K = s.K;
  fa.R = s.R;
  fa.Z = (uint32_t)s.Z;
  fa.W = (uint32_t)s.W;
  fa.d = (uint32_t)s.d;
  fa.vw = s.vs / 8;
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
  {
    TimedScope ts(m->timer, kkAccFetch, st);
    hipLaunchKernelGGL(k_acc_fetch, dim3((q + 3) / 4), dim3(256), 0, st, fa);
  }

  {
    TimedScope ts(m->timer, kkAccResolve, st);
    hipLaunchKernelGGL(k_acc_resolve, dim3((q + 255) / 256), dim3(256), 0, st, m->ctl, ops,
                       reinterpret_cast<const uint64_t*>(vals_in), bs.leader, bs.prevw, bs.found,
                       reinterpret_cast<const uint64_t*>(bs.fval), q, s.vs / 8, reinterpret_cast<uint64_t*>(vals_out),
                       status);
  }

  RemapArgs ra;
  ra.ctl = m->ctl;
  ra.ops = ops;
  ra.keys = keys;
  ra.vals_in = reinterpret_cast<const uint64_t*>(vals_in);
  ra.leader = bs.leader;
  ra.lastw = bs.lastw;
  ra.hit = bs.hit;
  ra.hrow = bs.hrow;
  ra.hslot = bs.hslot;
  ra.found = bs.found;
  ra.fval = reinterpret_cast<const uint64_t*>(bs.fval);
  ra.rpair = bs.rpair;
  ra.q = q;
  ra.epoch = epoch;
  ra.Z = (uint32_t)s.Z;
  ra.W = (uint32_t)s.W;
  ra.d = (uint32_t)s.d;
  ra.vw = s.vs / 8;
  ra.B = s.B;
  ra.K = s.K;
  ra.R = s.R;
  ra.P = s.P;
  ra.cap = s.cap;
  ra.load = m->load;
  ra.st_key = m->st_key;
  ra.st_val = reinterpret_cast<uint64_t*>(m->st_val);
  ra.st_dest = m->st_dest;
  ra.st_dead = m->st_dead;
  ra.ring = m->ring;
  ra.rev_cnt = m->rev_cnt;
  ra.rev_idx = m->rev_idx;
  ra.claim = m->claim;
  ra.cand_bin = bs.cand_bin;
  ra.pm_key = m->pm_key;
  ra.pm_pair = m->pm_pair;
  ra.pm_mask = m->pm_mask;
  {
    TimedScope ts(m->timer, kkAccRemap, st);
    hipLaunchKernelGGL(k_acc_remap, dim3(1), dim3(kRemapNT), 0, st, ra);
  }

  WbArgs wa;
  wa.ctl = m->ctl;
  wa.q = q;
  wa.epoch = epoch;
  wa.Z = (uint32_t)s.Z;
  wa.vw = s.vs / 8;
  wa.K = s.K;
  wa.P = s.P;
  wa.pw = s.page_bytes / 8;
  wa.cand_bin = bs.cand_bin;
  wa.claim = m->claim;
  wa.rmask = m->rmask;
  wa.stage = reinterpret_cast<uint64_t*>(bs.stage);
  wa.obs = reinterpret_cast<uint64_t*>(m->obs);
  wa.hbm = reinterpret_cast<uint64_t*>(m->hbm);
  wa.rev_cnt = m->rev_cnt;
  wa.rev_idx = m->rev_idx;
  wa.st_key = m->st_key;
  wa.st_val = reinterpret_cast<const uint64_t*>(m->st_val);
  wa.st_dead = m->st_dead;
  wa.ring = m->ring;
  wa.tlog_w = tlog_w;
  {
    TimedScope ts(m->timer, kkAccWriteback, st);
    hipLaunchKernelGGL(k_acc_writeback, dim3((3 * q + 3) / 4), dim3(256), 0, st, wa);
  }

  {
    TimedScope ts(m->timer, kkAccMisc, st);
    hipLaunchKernelGGL(k_acc_finish, dim3(1), dim3(64), 0, st, m->ctl, q, s.P, s.stash_bound);
  }
  m->batches++;
  return hipGetLastError() == hipSuccess ? BOLT_OK : BOLT_EHIP;
}

}  // namespace bolt
