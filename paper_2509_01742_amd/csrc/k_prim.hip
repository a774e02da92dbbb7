// Primitive kernels of the build path: PRF over an array, the bitonic
// sorting network (LDS tile stages + coalesced global stages), and the
// expansion (shift) network.  Every kernel here touches memory in an order
// that depends only on the array sizes.
#include "bolt_impl.h"

namespace bolt {

const char* const kKernelNames[kkCount] = {
    "sort_tile", "sort_global", "sort_merge", "build_pairs", "p2c_rounds", "loads_scan", "expand", "page_writeout",
    "pm_build", "dup_check", "build_misc", "acc_dedup", "acc_fetch", "acc_resolve", "acc_remap", "acc_compose",
    "acc_ship", "acc_misc", "acc_solo"};

hipEvent_t KernelTimer::take() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

void KernelTimer::begin(int id, hipStream_t st) {
  cur = id;
  cur_a = take();
  (void)hipEventRecord(cur_a, st);
}

void KernelTimer::end(hipStream_t st) {
  hipEvent_t b = take();
  (void)hipEventRecord(b, st);
  recs.push_back(Rec{cur, cur_a, b});
  cur = -1;
}

int KernelTimer::collect() {
  for (const Rec& r : recs) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return -1;
    total_ms[r.id] += ms;
    launches[r.id] += 1;
    pool.push_back(r.a);
    pool.push_back(r.b);
  }
  recs.clear();
  return 0;
}

void KernelTimer::reset() {
  for (int i = 0; i < kkCount; ++i) {
    total_ms[i] = 0;
    launches[i] = 0;
  }
}

KernelTimer::~KernelTimer() {
  for (const Rec& r : recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

// ---------------------------------------------------------------------------
// PRF
// ---------------------------------------------------------------------------

__global__ void k_prf_key_setup(Ctl* ctl, uint4 k0, uint4 k1) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  uint32_t kw[8] = {k0.x, k0.y, k0.z, k0.w, k1.x, k1.y, k1.z, k1.w};
  b2s_key_block(kw, ctl->hkey);
  uint32_t hk[8];
  for (int j = 0; j < 8; ++j) hk[j] = ctl->hkey[j];
  uint64_t w[4];
  prf4(hk, kDomSeal, 0, w);
  for (int j = 0; j < 4; ++j) {
    ctl->skey[2 * j] = (uint32_t)w[j];
    ctl->skey[2 * j + 1] = (uint32_t)(w[j] >> 32);
  }
}

__global__ void k_prf_array(const Ctl* ctl, uint32_t domain, const uint64_t* __restrict__ x, uint64_t n,
                            uint64_t* __restrict__ out) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t hk[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) hk[j] = ctl->hkey[j];
  uint64_t w[4];
  prf4(hk, domain, x[i], w);
  ulonglong2* o = reinterpret_cast<ulonglong2*>(out + 4 * i);
  o[0] = make_ulonglong2(w[0], w[1]);
  o[1] = make_ulonglong2(w[2], w[3]);
}

void launch_prf_key_setup(Ctl* ctl, const uint8_t key[32], hipStream_t st) {
  uint32_t kw[8];
  for (int i = 0; i < 8; ++i)
    kw[i] = (uint32_t)key[4 * i] | ((uint32_t)key[4 * i + 1] << 8) | ((uint32_t)key[4 * i + 2] << 16) |
            ((uint32_t)key[4 * i + 3] << 24);
  hipLaunchKernelGGL(k_prf_key_setup, dim3(1), dim3(64), 0, st, ctl, make_uint4(kw[0], kw[1], kw[2], kw[3]),
                     make_uint4(kw[4], kw[5], kw[6], kw[7]));
}

void launch_prf_array(const Ctl* ctl, uint32_t domain, const uint64_t* x, uint64_t n, uint64_t* out,
                      hipStream_t st) {
  if (n == 0) return;
  uint64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_prf_array, dim3((uint32_t)blocks), dim3(256), 0, st, ctl, domain, x, n, out);
}

// ---------------------------------------------------------------------------
// Bitonic sorting network.  Stage (k, j) compares element i with i + j
// (bit j of i clear); the pair sorts ascending when bit k of i is clear.
// Stages with j < T run in LDS on tiles of T elements; stages with j >= T run
// as global passes, F strides per pass, each thread holding 2^F elements in
// registers.
//
// Every kernel has a one-array form and a many-array form (MULTI): the
// latter sorts array blockIdx.y of a table, each of its own power-of-two
// length, with one launch per stage group for all of them.  The stage
// sequence of a length-2^L network is a prefix of that of any longer one,
// so an array simply sits out the stages past its own length.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void cmpex(uint64_t& x, uint64_t& y, bool asc) {
  uint64_t lo = x < y ? x : y;
  uint64_t hi = x < y ? y : x;
  x = asc ? lo : hi;
  y = asc ? hi : lo;
}


constexpr int kSortLogT = 13;  // largest tile: 8192 elements (64 KiB of LDS for the transposes)

// ---- tile of 8192 elements, 512 threads, 16 elements per thread --------
//
// Two register layouts of a tile: in the "row" layout thread t holds
// elements r * 512 + t (r = 0..15), so loads and stores are coalesced and
// the strides 512..4096 pair two registers of one thread; in the "column"
// layout thread t holds elements 16 t + r, so the strides 1..8 pair two
// registers and the strides 16..256 pair the same register of lanes
// 1..16 apart in one wave (exchanged by lane shuffles).  A stage therefore
// never touches LDS; LDS only transposes between the two layouts (with the
// low four index bits XOR-swizzled by the next four, so neither layout's
// accesses conflict on banks).  A full tile sort is 91 network stages and
// 10 transposes; the tail of a longer merge step is 13 stages and 2.

constexpr int kRegNT = 512;
constexpr int kRegE = 16;

__device__ __forceinline__ uint32_t tswz(uint32_t i) { return i ^ ((i >> 4) & 15u); }

// x := min(x, y) if takemin else max(x, y)
__device__ __forceinline__ uint64_t minmax(uint64_t x, uint64_t y, bool takemin) {
  return ((x < y) == takemin) ? x : y;
}

// Row -> column layout through LDS (and back).
__device__ __forceinline__ void rows_to_cols(uint64_t (&v)[kRegE], uint64_t* lds, uint32_t t) {
  __syncthreads();  // earlier readers of lds are done
#pragma unroll
  for (int r = 0; r < kRegE; ++r) lds[tswz((uint32_t)r * kRegNT + t)] = v[r];
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRegE; ++r) v[r] = lds[tswz(t * kRegE + (uint32_t)r)];
}

__device__ __forceinline__ void cols_to_rows(uint64_t (&v)[kRegE], uint64_t* lds, uint32_t t) {
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRegE; ++r) lds[tswz(t * kRegE + (uint32_t)r)] = v[r];
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRegE; ++r) v[r] = lds[tswz((uint32_t)r * kRegNT + t)];
}

// Direction of merge step K for an element whose index bits >= 4 are those
// of `hi` (base + 16 t in the column layout): ascending when bit K is clear.
template <int K>
__device__ __forceinline__ bool asc_of(uint64_t hi) {
  return ((hi >> K) & 1) == 0;
}

// Column layout, stride 2^JL with JL <= 3: registers r and r + 2^JL.
template <int K, int JL>
__device__ __forceinline__ void col_reg_stage(uint64_t (&v)[kRegE], uint64_t hi) {
  constexpr int m = 1 << JL;
#pragma unroll
  for (int r = 0; r < kRegE; ++r) {
    if (r & m) continue;
    bool asc;
    if constexpr (K <= 3)
      asc = ((r >> K) & 1) == 0;
    else
      asc = asc_of<K>(hi);
    const uint64_t x = v[r], y = v[r + m];
    v[r] = minmax(x, y, asc);
    v[r + m] = minmax(x, y, !asc);
  }
}

// The value of lane (lane XOR D), D in {1, 2, 4, 8, 16}: DPP quad
// permutations for 1 and 2 (plain VALU), the LDS crossbar's bit-mask
// swizzle (no LDS memory, no address operand) for 4, 8 and 16.
template <int D>
__device__ __forceinline__ uint32_t xor_lane32(uint32_t x) {
  if constexpr (D == 1)
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
  else if constexpr (D == 2)
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
  else
    return (uint32_t)__builtin_amdgcn_ds_swizzle((int)x, 0x1F | (D << 10));  // and 0x1F, or 0, xor D
}

template <int D>
__device__ __forceinline__ uint64_t xor_lane(uint64_t x) {
  const uint32_t lo = xor_lane32<D>((uint32_t)x), hi = xor_lane32<D>((uint32_t)(x >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Column layout, stride 2^JL with 4 <= JL <= 8: lanes 2^(JL-4) apart.
template <int K, int JL>
__device__ __forceinline__ void col_lane_stage(uint64_t (&v)[kRegE], uint64_t hi, uint32_t t) {
  constexpr int d = 1 << (JL - 4);
  const bool lower = ((t >> (JL - 4)) & 1) == 0;
  const bool takemin = lower == asc_of<K>(hi);
#pragma unroll
  for (int r = 0; r < kRegE; ++r) {
    const uint64_t y = xor_lane<d>(v[r]);
    v[r] = minmax(v[r], y, takemin);
  }
}

// Column layout: strides 2^JL .. 1 of merge step K.
template <int K, int JL>
__device__ __forceinline__ void col_stages(uint64_t (&v)[kRegE], uint64_t hi, uint32_t t) {
  if constexpr (JL >= 4)
    col_lane_stage<K, JL>(v, hi, t);
  else
    col_reg_stage<K, JL>(v, hi);
  if constexpr (JL > 0) col_stages<K, JL - 1>(v, hi, t);
}

// Row layout, stride 2^JL with 9 <= JL <= 12: registers r and r + 2^(JL-9).
// For K <= 12 the direction is bit K - 9 of r; above, bit K of the tile base.
template <int K, int JL>
__device__ __forceinline__ void row_stages(uint64_t (&v)[kRegE], uint64_t base) {
  constexpr int m = 1 << (JL - 9);
#pragma unroll
  for (int r = 0; r < kRegE; ++r) {
    if (r & m) continue;
    bool asc;
    if constexpr (K <= 12)
      asc = ((r >> (K - 9)) & 1) == 0;
    else
      asc = asc_of<K>(base);
    const uint64_t x = v[r], y = v[r + m];
    v[r] = minmax(x, y, asc);
    v[r + m] = minmax(x, y, !asc);
  }
  if constexpr (JL > 9) row_stages<K, JL - 1>(v, base);
}

// Merge steps K .. 9 of a full tile sort, all in the column layout.
template <int K>
__device__ __forceinline__ void tile_low_steps(uint64_t (&v)[kRegE], uint64_t hi, uint32_t t) {
  col_stages<K, K - 1>(v, hi, t);
  if constexpr (K < 9) tile_low_steps<K + 1>(v, hi, t);
}

// Merge steps K .. 13: long strides in rows, then the rest in columns.
template <int K>
__device__ __forceinline__ void tile_high_steps(uint64_t (&v)[kRegE], uint64_t* lds, uint64_t base, uint64_t hi,
                                                uint32_t t) {
  cols_to_rows(v, lds, t);
  row_stages<K, K - 1>(v, base);
  rows_to_cols(v, lds, t);
  col_stages<K, 8>(v, hi, t);
  if constexpr (K < 13) tile_high_steps<K + 1>(v, lds, base, hi, t);
}

// Full sort (mode 0) or the strides 4096 .. 1 of merge step k_log > 13
// (mode 1) of the 8192-element tile at `base`.
__device__ __forceinline__ void tile_sort_regs(uint64_t* __restrict__ a, uint64_t base, int mode, uint32_t k_log,
                                               uint64_t* lds) {
  const uint32_t t = threadIdx.x;
  // one uniform tile pointer and 32-bit element offsets: each load and store
  // needs one offset register, not a 64-bit address
  char* __restrict__ tile = reinterpret_cast<char*>(a + base);
  const uint32_t tb = t * 8u;  // byte offset of register 0
  uint64_t v[kRegE];
#pragma unroll
  for (int r = 0; r < kRegE; ++r) v[r] = *reinterpret_cast<const uint64_t*>(tile + (tb + (uint32_t)r * kRegNT * 8u));
  const uint64_t hi = base + (uint64_t)t * kRegE;
  if (mode == 0) {
    rows_to_cols(v, lds, t);
    tile_low_steps<1>(v, hi, t);
    tile_high_steps<10>(v, lds, base, hi, t);
  } else {
    // one step k_log > 13: the direction is bit k_log of base for the whole tile
    const bool asc = ((base >> k_log) & 1) == 0;
    const uint64_t h = asc ? 0 : (1ull << 14);  // a stand-in whose bit 14 carries the direction
    row_stages<14, 12>(v, h);
    rows_to_cols(v, lds, t);
    col_stages<14, 8>(v, h, t);
  }
  cols_to_rows(v, lds, t);
  // An empty register constraint on the offset: the store addresses are
  // formed here, not kept live (and spilled) since the loads.
  uint32_t tb2 = tb;
  asm volatile("" : "+v"(tb2));
#pragma unroll
  for (int r = 0; r < kRegE; ++r) *reinterpret_cast<uint64_t*>(tile + (tb2 + (uint32_t)r * kRegNT * 8u)) = v[r];
}

// LDS stages on one tile of T = 2^logt <= 8192 elements, one stage per
// pass (tiles shorter than 8192: arrays below 8192 elements).  Mode 0: full
// tile sort.  Mode 1: the tail of merge step k (strides T/2 .. 1).
__device__ __forceinline__ void tile_sort_lds(uint64_t* __restrict__ a, uint64_t base, uint32_t logt, int mode,
                                              uint32_t k_log, uint64_t* s) {
  const uint32_t T = 1u << logt;
  for (uint32_t x = threadIdx.x; x < T; x += kRegNT) s[x] = a[base + x];
  __syncthreads();
  const uint32_t half = T >> 1;
  const uint32_t kl0 = mode == 0 ? 1 : logt;
  for (uint32_t kl = kl0; kl <= logt; ++kl) {
    for (int jl = (int)kl - 1; jl >= 0; --jl) {
      const uint32_t j = 1u << jl;
      for (uint32_t p = threadIdx.x; p < half; p += kRegNT) {
        uint32_t i = ((p >> jl) << (jl + 1)) | (p & (j - 1));
        const uint32_t kk = mode == 0 ? kl : k_log;
        bool asc = (((base + i) >> kk) & 1) == 0;
        uint64_t x = s[i], y = s[i + j];
        cmpex(x, y, asc);
        s[i] = x;
        s[i + j] = y;
      }
      __syncthreads();
    }
  }
  for (uint32_t x = threadIdx.x; x < T; x += kRegNT) a[base + x] = s[x];
}

// One launch of the tile stages: 8192-element tiles in registers, shorter
// (whole-array) tiles in LDS.
template <bool MULTI>
__global__ __launch_bounds__(kRegNT, 4) void k_bitonic_tile(uint64_t* __restrict__ a1, uint32_t logt1, int mode,
                                                         uint32_t k_log, const NetSeg* segs) {
  __shared__ uint64_t lds[1 << kSortLogT];
  uint64_t* __restrict__ a = a1;
  uint32_t logt = logt1;
  if (MULTI) {
    const NetSeg g = segs[blockIdx.y];
    const uint32_t L = ilog2_ceil(g.n);
    if (mode == 1 && L < k_log) return;  // whole block: this array is shorter
    logt = L < logt1 ? L : logt1;  // logt1: the schedule's tile (at most kSortLogT)
    if (blockIdx.x >= (g.n >> logt)) return;
    a = g.a;
  }
  const uint64_t base = (uint64_t)blockIdx.x << logt;
  if (logt == (uint32_t)kSortLogT)
    tile_sort_regs(a, base, mode, k_log, lds);
  else
    tile_sort_lds(a, base, logt, mode, k_log, lds);
}

// F consecutive strides 2^(jl_top) .. 2^(jl_top - F + 1) of merge step k in
// one pass over the array.
template <int F, bool MULTI>
__global__ __launch_bounds__(256) void k_bitonic_global(uint64_t* __restrict__ a1, uint64_t n1, uint32_t k_log,
                                                        uint32_t jl_top, const NetSeg* segs) {
  uint64_t* __restrict__ a = a1;
  uint64_t n = n1;
  if (MULTI) {
    const NetSeg g = segs[blockIdx.y];
    if (ilog2_ceil(g.n) < k_log) return;
    a = g.a;
    n = g.n;
  }
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (n >> F)) return;
  const uint32_t low = jl_top - F + 1;
  const uint64_t lowmask = (1ull << low) - 1;
  const uint64_t i0 = (t & lowmask) | ((t >> low) << (low + F));
  const bool asc = ((i0 >> k_log) & 1) == 0;
  uint64_t e[1 << F];
  // non-temporal loads and stores: each element is touched once per pass,
  // and keeping the stream out of the caches measured 9 % faster at 2^26
#pragma unroll
  for (int x = 0; x < (1 << F); ++x) e[x] = __builtin_nontemporal_load(a + i0 + ((uint64_t)x << low));
#pragma unroll
  for (int f = F - 1; f >= 0; --f) {
#pragma unroll
    for (int x = 0; x < (1 << F); ++x)
      if (!(x & (1 << f))) cmpex(e[x], e[x | (1 << f)], asc);
  }
#pragma unroll
  for (int x = 0; x < (1 << F); ++x) __builtin_nontemporal_store(e[x], a + i0 + ((uint64_t)x << low));
}

// One sort schedule for one array (segs == nullptr) or for `count` arrays
// of the device table `segs` whose longest has length nmax: tiles of
// 2^tile_log elements (11..13; 13 runs in registers), then up to fmax
// (1..6) strides per global pass.  Every choice sorts the same way.
template <bool MULTI>
static void sort_schedule(uint64_t* a, uint64_t nmax, const NetSeg* segs, uint32_t count, hipStream_t st,
                          KernelTimer* tm, uint32_t tile_log, uint32_t fmax) {
  if (nmax < 2) return;
  const uint32_t L = ilog2_ceil(nmax);
  const uint32_t logt = L < tile_log ? L : tile_log;
  const uint64_t tiles = nmax >> logt;
  {
    TimedScope ts(tm, kkSortTile, st);
    hipLaunchKernelGGL((k_bitonic_tile<MULTI>), dim3((uint32_t)tiles, count), dim3(kRegNT), 0, st, a, logt, 0, 0u,
                       segs);
  }
  for (uint32_t k_log = logt + 1; k_log <= L; ++k_log) {
    int jl = (int)k_log - 1;
    while (jl >= (int)logt) {
      int F = jl - (int)logt + 1;
      if (F > (int)fmax) F = (int)fmax;
      TimedScope ts(tm, kkSortGlobal, st);
      const dim3 grid((uint32_t)(((nmax >> F) + 255) / 256), count), block(256);
      switch (F) {
        case 1: hipLaunchKernelGGL((k_bitonic_global<1, MULTI>), grid, block, 0, st, a, nmax, k_log, (uint32_t)jl, segs); break;
        case 2: hipLaunchKernelGGL((k_bitonic_global<2, MULTI>), grid, block, 0, st, a, nmax, k_log, (uint32_t)jl, segs); break;
        case 3: hipLaunchKernelGGL((k_bitonic_global<3, MULTI>), grid, block, 0, st, a, nmax, k_log, (uint32_t)jl, segs); break;
        case 4: hipLaunchKernelGGL((k_bitonic_global<4, MULTI>), grid, block, 0, st, a, nmax, k_log, (uint32_t)jl, segs); break;
        case 5: hipLaunchKernelGGL((k_bitonic_global<5, MULTI>), grid, block, 0, st, a, nmax, k_log, (uint32_t)jl, segs); break;
        default: hipLaunchKernelGGL((k_bitonic_global<6, MULTI>), grid, block, 0, st, a, nmax, k_log, (uint32_t)jl, segs); break;
      }
      jl -= F;
    }
    TimedScope ts(tm, kkSortMerge, st);
    hipLaunchKernelGGL((k_bitonic_tile<MULTI>), dim3((uint32_t)tiles, count), dim3(kRegNT), 0, st, a, logt, 1,
                       k_log, segs);
  }
}

void launch_bitonic_sort(uint64_t* a, uint64_t n, hipStream_t st, KernelTimer* tm) {
  const NetTune t = net_tune(ilog2_ceil(n));
  sort_schedule<false>(a, n, nullptr, 1, st, tm, t.sort_tile_log, t.sort_fmax);
}

void launch_bitonic_sort_with(uint64_t* a, uint64_t n, hipStream_t st, uint32_t tile_log, uint32_t fmax) {
  sort_schedule<false>(a, n, nullptr, 1, st, nullptr, tile_log, fmax);
}

void launch_bitonic_sort_many(const NetSeg* segs, uint32_t count, uint64_t nmax, hipStream_t st) {
  const NetTune t = net_tune(ilog2_ceil(nmax));
  if (count) sort_schedule<true>(nullptr, nmax, segs, count, st, nullptr, t.sort_tile_log, t.sort_fmax);
}

// ---------------------------------------------------------------------------
// Expansion network.  Element = (target << 32 | payload); all ones = empty.
// Stage j moves an element right by 2^j when bit j of (target - position)
// is set; each output position reads both candidates (stay / arrive), so
// the memory accesses depend only on m.
//
// Stages run from the top bit down.  The stages with stride >= 2^kExpLow run
// as global passes, F of them per pass: along one residue class modulo the
// group's lowest stride the F stages are a small expansion network over
// consecutive coordinates, so a thread pulls 2F - 1 ... (2^(F+1) - 1)
// elements of its strip into registers and emits the last 2^F.  The stages
// below 2^kExpLow then run in LDS on tiles of kExpTile outputs, each tile
// loading the kExpHalo elements to its left (no element moves further than
// 2^kExpLow - 1 in those stages).
//
// A stage with 2^j >= m is the identity (target - position < m), so the
// many-array form runs the longest array's stages on every array.  Passes
// alternate between an array and its scratch; `flip` says which way.
// ---------------------------------------------------------------------------

constexpr int kExpLow = 10;
static_assert(kExpLow >= 8, "the fused expansion passes take whole workgroups of 256 residues");
constexpr uint32_t kExpTile = 4096;
constexpr uint32_t kExpHalo = 1u << kExpLow;

__device__ __forceinline__ uint64_t exp_step(uint64_t cur, uint64_t prev, uint64_t pos, uint64_t h) {
  const bool stay = cur != kNone64 && !(((cur >> 32) - pos) & h);
  const bool arrive = prev != kNone64 && pos >= h && (((prev >> 32) - (pos - h)) & h);
  return stay ? cur : (arrive ? prev : kNone64);
}

template <bool MULTI>
__device__ __forceinline__ bool exp_pick(const NetSeg* segs, uint32_t flip, const uint64_t*& in, uint64_t*& out,
                                         uint64_t& m) {
  if (!MULTI) return true;
  const NetSeg g = segs[blockIdx.y];
  in = flip ? g.b : g.a;
  out = flip ? g.a : g.b;
  m = g.n;
  return m >= 1;  // a one-element array is copied through unchanged
}

// Stages jlow + F - 1 .. jlow in one pass.  Coordinate c is position
// c * 2^jlow + r for residue r.  A wave takes 64 consecutive residues and a
// group of 2^F consecutive coordinates (its outputs); it also needs the
// 2^F - 1 coordinates to the left (elements arriving from there).  With
// `share` (four groups or more), the four waves of a workgroup take four
// consecutive groups of the same residues, so each wave hands the inputs of
// its last 2^F - 1 coordinates to the next wave through LDS and only wave 0
// loads its left part from memory: the pass reads about 1.2 times what it
// writes instead of 2.  Without (the top passes, fewer groups than waves),
// the four waves take four consecutive residue chunks of one group and load
// their own left parts.  2^jlow >= 256: whole workgroups of residues.
template <int F, bool MULTI>
__global__ __launch_bounds__(256) void k_expand_fused(const uint64_t* __restrict__ in1, uint64_t* __restrict__ out1,
                                                      uint64_t m1, uint32_t jlow, const NetSeg* segs, uint32_t flip,
                                                      uint32_t share) {
  const uint64_t* in = in1;
  uint64_t* out = out1;
  uint64_t m = m1;
  if (!exp_pick<MULTI>(segs, flip, in, out, m)) return;  // whole block
  constexpr int NB = 1 << F;      // outputs per thread
  constexpr int NW = 2 * NB - 1;  // window: NB - 1 to the left
  __shared__ uint64_t halo[3][NB - 1][64];
  const uint64_t hl = 1ull << jlow;
  const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t rchunks = hl >> 6;
  uint64_t r, c0;
  if (share) {
    r = (blockIdx.x % rchunks) * 64 + lane;
    c0 = ((blockIdx.x / rchunks) * 4 + w) * NB;
  } else {
    const uint64_t rq = rchunks >> 2;
    r = ((blockIdx.x % rq) * 4 + w) * 64 + lane;
    c0 = (blockIdx.x / rq) * NB;
  }
  const uint64_t ncoord = (m + hl - 1) >> jlow;
  const bool act = c0 < ncoord && r < m;  // no return before the barrier
  uint64_t v[NW];
#pragma unroll
  for (int k = NB - 1; k < NW; ++k) {
    const uint64_t pos = (c0 + (k - (NB - 1))) * hl + r;
    v[k] = (act && pos < m) ? in[pos] : kNone64;
  }
  if (share && w < 3) {
#pragma unroll
    for (int j = 0; j < NB - 1; ++j) halo[w][j][lane] = v[NB + j];
  }
  if (!share || w == 0) {
#pragma unroll
    for (int k = 0; k < NB - 1; ++k) {
      const int64_t c = (int64_t)c0 - (NB - 1) + k;
      const uint64_t pos = (uint64_t)c * hl + r;
      v[k] = (act && c >= 0 && pos < m) ? in[pos] : kNone64;
    }
  }
  __syncthreads();
  if (share && w > 0) {
    // the previous wave's coordinates c0 - NB + 1 .. c0 - 1 (it is active
    // whenever this one is: same residues, lower coordinates)
#pragma unroll
    for (int k = 0; k < NB - 1; ++k) v[k] = halo[w - 1][k][lane];
  }
  if (!act) return;
#pragma unroll
  for (int f = F - 1; f >= 0; --f) {
    const int d = 1 << f;
    const uint64_t h = hl << f;
#pragma unroll
    for (int k = NW - 1; k >= 0; --k) {  // descending: v[k - d] is still the old value
      const int64_t c = (int64_t)c0 - (NB - 1) + k;
      const uint64_t pos = (uint64_t)c * hl + r;
      const uint64_t prev = k >= d ? v[k - d] : kNone64;
      v[k] = c >= 0 ? exp_step(v[k], prev, pos, h) : kNone64;
    }
  }
#pragma unroll
  for (int k = NB - 1; k < NW; ++k) {
    const uint64_t pos = (c0 + (k - (NB - 1))) * hl + r;
    if (pos < m) out[pos] = v[k];
  }
}

// Stages jtop .. 0 (jtop < kExpLow) on LDS tiles with a left halo.
template <bool MULTI>
__global__ __launch_bounds__(1024) void k_expand_tile(const uint64_t* __restrict__ in1, uint64_t* __restrict__ out1,
                                                     uint64_t m1, int jtop, const NetSeg* segs, uint32_t flip) {
  const uint64_t* in = in1;
  uint64_t* out = out1;
  uint64_t m = m1;
  if (!exp_pick<MULTI>(segs, flip, in, out, m)) return;
  const uint64_t p0 = (uint64_t)blockIdx.x * kExpTile;
  if (p0 >= m) return;  // whole block
  __shared__ uint64_t A[kExpTile + kExpHalo];
  __shared__ uint64_t Bf[kExpTile + kExpHalo];
  constexpr uint32_t NWIN = kExpTile + kExpHalo;
  for (uint32_t x = threadIdx.x; x < NWIN; x += 1024) {
    const int64_t pos = (int64_t)p0 - (int64_t)kExpHalo + x;
    A[x] = (pos >= 0 && (uint64_t)pos < m) ? in[pos] : kNone64;
  }
  __syncthreads();
  uint64_t* cur = A;
  uint64_t* nxt = Bf;
  for (int j = jtop; j >= 0; --j) {
    const uint32_t h = 1u << j;
    for (uint32_t x = threadIdx.x; x < NWIN; x += 1024) {
      const int64_t pos = (int64_t)p0 - (int64_t)kExpHalo + x;
      const uint64_t prev = x >= h ? cur[x - h] : kNone64;
      nxt[x] = pos >= 0 ? exp_step(cur[x], prev, (uint64_t)pos, h) : kNone64;
    }
    __syncthreads();
    uint64_t* t = cur;
    cur = nxt;
    nxt = t;
  }
  for (uint32_t x = threadIdx.x; x < kExpTile; x += 1024) {
    const uint64_t pos = p0 + x;
    if (pos < m) out[pos] = cur[kExpHalo + x];
  }
}

// Runs every stage for one array (segs == nullptr: a / tmp of length mmax)
// or for the arrays of a device table.  Returns true when the result ended
// in the scratch buffer (tmp, or each entry's b).
template <bool MULTI>
static bool expand_schedule(uint64_t* a, uint64_t* tmp, uint64_t mmax, const NetSeg* segs, uint32_t count,
                            hipStream_t st, KernelTimer* tm, uint32_t fmax) {
  if (mmax < 2) return false;
  int top = 0;
  while ((2ull << top) <= mmax - 1) ++top;
  uint64_t* src = a;
  uint64_t* dst = tmp;
  uint32_t flip = 0;
  int j = top;
  while (j >= kExpLow) {  // global passes, up to 4 stages each
    int F = j - kExpLow + 1;
    if (F > (int)fmax) F = (int)fmax;
    TimedScope ts(tm, kkExpand, st);
    const uint32_t jlow = (uint32_t)(j - F + 1);
    const uint64_t hl = 1ull << jlow;  // >= 2^kExpLow: whole workgroups of residues
    const uint64_t ncoord = (mmax + hl - 1) >> jlow;
    const uint64_t groups = (ncoord + (1u << F) - 1) >> F;  // of 2^F coordinates
    const uint32_t share = groups >= 4 ? 1 : 0;  // four groups per workgroup, else four residue chunks
    const uint64_t blocks = share ? ((groups + 3) / 4) * (hl >> 6) : groups * (hl >> 8);
    const dim3 grid((uint32_t)blocks, count), block(256);
    switch (F) {
      case 1: hipLaunchKernelGGL((k_expand_fused<1, MULTI>), grid, block, 0, st, src, dst, mmax, jlow, segs, flip, share); break;
      case 2: hipLaunchKernelGGL((k_expand_fused<2, MULTI>), grid, block, 0, st, src, dst, mmax, jlow, segs, flip, share); break;
      case 3: hipLaunchKernelGGL((k_expand_fused<3, MULTI>), grid, block, 0, st, src, dst, mmax, jlow, segs, flip, share); break;
      default: hipLaunchKernelGGL((k_expand_fused<4, MULTI>), grid, block, 0, st, src, dst, mmax, jlow, segs, flip, share); break;
    }
    uint64_t* t = src;
    src = dst;
    dst = t;
    flip ^= 1;
    j -= F;
  }
  {  // the low stages on LDS tiles
    TimedScope ts(tm, kkExpand, st);
    hipLaunchKernelGGL((k_expand_tile<MULTI>), dim3((uint32_t)((mmax + kExpTile - 1) / kExpTile), count), dim3(1024),
                       0, st, src, dst, mmax, j, segs, flip);
    flip ^= 1;
  }
  return flip != 0;
}

uint64_t* launch_expand_inplace(uint64_t* a, uint64_t* tmp, uint64_t m, hipStream_t st, KernelTimer* tm) {
  return expand_schedule<false>(a, tmp, m, nullptr, 1, st, tm, net_tune(ilog2_ceil(m)).exp_fmax) ? tmp : a;
}

void launch_expand(uint64_t* a, uint64_t* tmp, uint64_t m, hipStream_t st, KernelTimer* tm) {
  uint64_t* r = launch_expand_inplace(a, tmp, m, st, tm);
  if (r != a) (void)hipMemcpyAsync(a, r, m * sizeof(uint64_t), hipMemcpyDeviceToDevice, st);
}

bool launch_expand_many(const NetSeg* segs, uint32_t count, uint64_t mmax, hipStream_t st) {
  return count ? expand_schedule<true>(nullptr, nullptr, mmax, segs, count, st, nullptr,
                                       net_tune(ilog2_ceil(mmax)).exp_fmax)
               : false;
}

uint64_t* launch_expand_with(uint64_t* a, uint64_t* tmp, uint64_t m, hipStream_t st, uint32_t fmax) {
  return expand_schedule<false>(a, tmp, m, nullptr, 1, st, nullptr, fmax) ? tmp : a;
}

}  // namespace bolt
