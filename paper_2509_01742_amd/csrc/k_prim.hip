// Primitive kernels of the build path: PRF over an array, the bitonic
// sorting network (LDS tile stages + coalesced global stages), and the
// expansion (shift) network.  Every kernel here touches memory in an order
// that depends only on the array sizes.
#include "bolt_impl.h"

namespace bolt {

const char* const kKernelNames[kkCount] = {
    "sort_tile", "sort_global", "sort_merge", "build_pairs", "p2c_rounds", "loads_scan", "expand", "page_writeout",
    "pm_build", "dup_check", "build_misc", "acc_dedup", "acc_fetch", "acc_resolve", "acc_remap", "acc_writeback",
    "acc_misc"};

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
// ---------------------------------------------------------------------------

__device__ __forceinline__ void cmpex(uint64_t& x, uint64_t& y, bool asc) {
  uint64_t lo = x < y ? x : y;
  uint64_t hi = x < y ? y : x;
  x = asc ? lo : hi;
  y = asc ? hi : lo;
}

// LDS stages on one tile.  Mode 0: full tile sort, k = 2 .. T.  Mode 1: the
// tail of merge step k (strides T/2 .. 1).
template <int LOGT, int NT>
__global__ __launch_bounds__(NT) void k_bitonic_tile(uint64_t* __restrict__ a, uint32_t logt, int mode,
                                                     uint32_t k_log) {
  __shared__ uint64_t s[1 << LOGT];
  const uint32_t T = 1u << logt;
  const uint64_t base = (uint64_t)blockIdx.x * T;
  for (uint32_t x = threadIdx.x; x < T; x += NT) s[x] = a[base + x];
  __syncthreads();
  const uint32_t half = T >> 1;
  if (mode == 0) {
    for (uint32_t kl = 1; kl <= logt; ++kl) {
      for (int jl = (int)kl - 1; jl >= 0; --jl) {
        const uint32_t j = 1u << jl;
        for (uint32_t p = threadIdx.x; p < half; p += NT) {
          uint32_t i = ((p >> jl) << (jl + 1)) | (p & (j - 1));
          bool asc = (((base + i) >> kl) & 1) == 0;
          uint64_t x = s[i], y = s[i + j];
          cmpex(x, y, asc);
          s[i] = x;
          s[i + j] = y;
        }
        __syncthreads();
      }
    }
  } else {
    const bool asc = ((base >> k_log) & 1) == 0;
    for (int jl = (int)logt - 1; jl >= 0; --jl) {
      const uint32_t j = 1u << jl;
      for (uint32_t p = threadIdx.x; p < half; p += NT) {
        uint32_t i = ((p >> jl) << (jl + 1)) | (p & (j - 1));
        uint64_t x = s[i], y = s[i + j];
        cmpex(x, y, asc);
        s[i] = x;
        s[i + j] = y;
      }
      __syncthreads();
    }
  }
  for (uint32_t x = threadIdx.x; x < T; x += NT) a[base + x] = s[x];
}

// F consecutive strides 2^(jl_top) .. 2^(jl_top - F + 1) of merge step k in
// one pass over the array.
template <int F>
__global__ __launch_bounds__(256) void k_bitonic_global(uint64_t* __restrict__ a, uint64_t n, uint32_t k_log,
                                                        uint32_t jl_top) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (n >> F)) return;
  const uint32_t low = jl_top - F + 1;
  const uint64_t lowmask = (1ull << low) - 1;
  const uint64_t i0 = (t & lowmask) | ((t >> low) << (low + F));
  const bool asc = ((i0 >> k_log) & 1) == 0;
  uint64_t e[1 << F];
#pragma unroll
  for (int x = 0; x < (1 << F); ++x) e[x] = a[i0 + ((uint64_t)x << low)];
#pragma unroll
  for (int f = F - 1; f >= 0; --f) {
#pragma unroll
    for (int x = 0; x < (1 << F); ++x)
      if (!(x & (1 << f))) cmpex(e[x], e[x | (1 << f)], asc);
  }
#pragma unroll
  for (int x = 0; x < (1 << F); ++x) a[i0 + ((uint64_t)x << low)] = e[x];
}

constexpr int kSortLogT = 13;  // 8192-element LDS tiles (64 KiB)
constexpr int kSortNT = 1024;
constexpr int kSortFMax = 4;

static uint32_t ilog2(uint64_t n) {
  uint32_t l = 0;
  while ((1ull << l) < n) ++l;
  return l;
}

static void launch_global(uint64_t* a, uint64_t n, uint32_t k_log, uint32_t jl_top, int F, hipStream_t st,
                          KernelTimer* tm) {
  TimedScope ts(tm, kkSortGlobal, st);
  uint64_t threads = n >> F;
  dim3 grid((uint32_t)((threads + 255) / 256)), block(256);
  switch (F) {
    case 1: hipLaunchKernelGGL(k_bitonic_global<1>, grid, block, 0, st, a, n, k_log, jl_top); break;
    case 2: hipLaunchKernelGGL(k_bitonic_global<2>, grid, block, 0, st, a, n, k_log, jl_top); break;
    case 3: hipLaunchKernelGGL(k_bitonic_global<3>, grid, block, 0, st, a, n, k_log, jl_top); break;
    default: hipLaunchKernelGGL(k_bitonic_global<4>, grid, block, 0, st, a, n, k_log, jl_top); break;
  }
}

void launch_bitonic_sort(uint64_t* a, uint64_t n, hipStream_t st, KernelTimer* tm) {
  if (n < 2) return;
  const uint32_t L = ilog2(n);
  const uint32_t logt = L < (uint32_t)kSortLogT ? L : (uint32_t)kSortLogT;
  const uint64_t tiles = n >> logt;
  {
    TimedScope ts(tm, kkSortTile, st);
    hipLaunchKernelGGL((k_bitonic_tile<kSortLogT, kSortNT>), dim3((uint32_t)tiles), dim3(kSortNT), 0, st, a, logt, 0,
                       0u);
  }
  for (uint32_t k_log = logt + 1; k_log <= L; ++k_log) {
    int jl = (int)k_log - 1;
    while (jl >= (int)logt) {
      int F = jl - (int)logt + 1;
      if (F > kSortFMax) F = kSortFMax;
      launch_global(a, n, k_log, (uint32_t)jl, F, st, tm);
      jl -= F;
    }
    TimedScope ts(tm, kkSortMerge, st);
    hipLaunchKernelGGL((k_bitonic_tile<kSortLogT, kSortNT>), dim3((uint32_t)tiles), dim3(kSortNT), 0, st, a, logt,
                       1, k_log);
  }
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
// ---------------------------------------------------------------------------

constexpr int kExpLow = 10;
constexpr uint32_t kExpTile = 4096;
constexpr uint32_t kExpHalo = 1u << kExpLow;

__device__ __forceinline__ uint64_t exp_step(uint64_t cur, uint64_t prev, uint64_t pos, uint64_t h) {
  const bool stay = cur != kNone64 && !(((cur >> 32) - pos) & h);
  const bool arrive = prev != kNone64 && pos >= h && (((prev >> 32) - (pos - h)) & h);
  return stay ? cur : (arrive ? prev : kNone64);
}

// One stage per pass (used for m too small for the fused forms).
__global__ void k_expand_stage(const uint64_t* __restrict__ in, uint64_t* __restrict__ out, uint64_t m, uint32_t j) {
  uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= m) return;
  const uint64_t h = 1ull << j;
  out[p] = exp_step(in[p], p >= h ? in[p - h] : kNone64, p, h);
}

// Stages jlow + F - 1 .. jlow in one pass.  Thread = (residue r, block of
// 2^F coordinates c0..); coordinate c is position c * 2^jlow + r.
template <int F>
__global__ __launch_bounds__(256) void k_expand_fused(const uint64_t* __restrict__ in, uint64_t* __restrict__ out,
                                                      uint64_t m, uint32_t jlow) {
  constexpr int NB = 1 << F;      // outputs per thread
  constexpr int NW = 2 * NB - 1;  // window: NB - 1 to the left
  const uint64_t hl = 1ull << jlow;
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t r = t & (hl - 1);
  const uint64_t c0 = (t >> jlow) * NB;
  const uint64_t ncoord = (m + hl - 1) >> jlow;
  if (c0 >= ncoord) return;
  uint64_t v[NW];
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    const int64_t c = (int64_t)c0 - (NB - 1) + k;
    const uint64_t pos = (uint64_t)c * hl + r;
    v[k] = (c >= 0 && pos < m) ? in[pos] : kNone64;
  }
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
__global__ __launch_bounds__(1024) void k_expand_tile(const uint64_t* __restrict__ in, uint64_t* __restrict__ out,
                                                     uint64_t m, int jtop) {
  __shared__ uint64_t A[kExpTile + kExpHalo];
  __shared__ uint64_t Bf[kExpTile + kExpHalo];
  const uint64_t p0 = (uint64_t)blockIdx.x * kExpTile;
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

static void launch_fused(const uint64_t* in, uint64_t* out, uint64_t m, uint32_t jlow, int F, hipStream_t st) {
  const uint64_t hl = 1ull << jlow;
  const uint64_t ncoord = (m + hl - 1) >> jlow;
  const uint64_t threads = ((ncoord + (1u << F) - 1) >> F) * hl;
  dim3 grid((uint32_t)((threads + 255) / 256)), block(256);
  switch (F) {
    case 1: hipLaunchKernelGGL(k_expand_fused<1>, grid, block, 0, st, in, out, m, jlow); break;
    case 2: hipLaunchKernelGGL(k_expand_fused<2>, grid, block, 0, st, in, out, m, jlow); break;
    case 3: hipLaunchKernelGGL(k_expand_fused<3>, grid, block, 0, st, in, out, m, jlow); break;
    default: hipLaunchKernelGGL(k_expand_fused<4>, grid, block, 0, st, in, out, m, jlow); break;
  }
}

// Runs all stages; the result ends in `a` (tmp is scratch of m elements).
void launch_expand(uint64_t* a, uint64_t* tmp, uint64_t m, hipStream_t st, KernelTimer* tm) {
  if (m < 2) return;
  int top = 0;
  while ((2ull << top) <= m - 1) ++top;
  uint64_t* src = a;
  uint64_t* dst = tmp;
  int j = top;
  while (j >= kExpLow) {  // global passes, up to 4 stages each
    int F = j - kExpLow + 1;
    if (F > 4) F = 4;
    TimedScope ts(tm, kkExpand, st);
    launch_fused(src, dst, m, (uint32_t)(j - F + 1), F, st);
    uint64_t* t = src;
    src = dst;
    dst = t;
    j -= F;
  }
  {  // the low stages on LDS tiles
    TimedScope ts(tm, kkExpand, st);
    hipLaunchKernelGGL(k_expand_tile, dim3((uint32_t)((m + kExpTile - 1) / kExpTile)), dim3(1024), 0, st, src, dst, m,
                       j);
    uint64_t* t = src;
    src = dst;
    dst = t;
  }
  if (src != a) (void)hipMemcpyAsync(a, src, m * sizeof(uint64_t), hipMemcpyDeviceToDevice, st);
}

}  // namespace bolt
