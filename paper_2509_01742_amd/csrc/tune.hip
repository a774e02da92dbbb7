// Autotuner of the network schedules (sort tile, strides per global sort
// pass, stages per global expansion pass), per array-length class and
// device.  Each candidate runs on the device on a scratch array of the
// class's length and is timed with HIP events; the fastest is kept for the
// process and, given a path, written to (or read back from) a cache file.
// The choices change no result, and the memory access pattern of every
// network still depends on the array length alone.
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "bolt_impl.h"

using namespace bolt;

namespace {

constexpr int kMaxDev = 16;
constexpr uint32_t kMaxLog = 40;
constexpr uint32_t kTuneMinLog = 14;  // shorter arrays keep the defaults
constexpr uint32_t kTuneMaxLog = 28;
constexpr uint32_t kSortFMax = 6;  // strides per global sort pass: 1..6
constexpr uint32_t kExpFMax = 4;   // stages per global expansion pass: 1..4

struct Entry {
  NetTune t{13, 4, 4};
  float sort_ms = 0, exp_ms = 0;
  bool tuned = false;
};

std::mutex g_mu;
Entry g_tab[kMaxDev][kMaxLog + 1];

int cur_dev() {
  int d = 0;
  if (hipGetDevice(&d) != hipSuccess || d < 0 || d >= kMaxDev) d = 0;
  return d;
}

std::string dev_name(int d) {
  hipDeviceProp_t pr;
  if (hipGetDeviceProperties(&pr, d) != hipSuccess) return "unknown";
  std::string n = pr.gcnArchName;
  n += "/";
  n += std::to_string(pr.multiProcessorCount);
  for (char& c : n)
    if (c == ' ' || c == '\n') c = '_';
  return n;
}

__global__ void k_tune_fill(uint64_t* a, uint64_t n, uint32_t kind) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (kind == 0) {  // sort input: a SplitMix64-style hash of the position
    uint64_t x = i + 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    a[i] = x ^ (x >> 31);
  } else {  // expansion input: half the positions hold an element at its own target
    a[i] = i < n / 2 ? ((i << 32) | (uint32_t)i) : kNone64;
  }
}

bool load_cache(const char* path, int dev) {
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char name[256];
  bool ok = fscanf(f, "bolt-tune 1 %255s\n", name) == 1 && dev_name(dev) == name;
  std::vector<std::pair<uint32_t, Entry>> got;
  while (ok) {
    unsigned L, tl, fs, fe;
    float sm, em;
    const int r = fscanf(f, "%u %u %u %u %f %f\n", &L, &tl, &fs, &fe, &sm, &em);
    if (r == EOF) break;
    if (r != 6 || L > kMaxLog || tl < 11 || tl > 13 || fs < 1 || fs > kSortFMax || fe < 1 || fe > kExpFMax) {
      ok = false;
      break;
    }
    Entry e;
    e.t = NetTune{tl, fs, fe};
    e.sort_ms = sm;
    e.exp_ms = em;
    e.tuned = true;
    got.push_back({L, e});
  }
  fclose(f);
  if (!ok || got.empty()) return false;
  std::lock_guard<std::mutex> g(g_mu);
  for (auto& kv : got) g_tab[dev][kv.first] = kv.second;
  return true;
}

bool save_cache(const char* path, int dev) {
  FILE* f = fopen(path, "w");
  if (!f) return false;
  fprintf(f, "bolt-tune 1 %s\n", dev_name(dev).c_str());
  std::lock_guard<std::mutex> g(g_mu);
  for (uint32_t L = 0; L <= kMaxLog; ++L) {
    const Entry& e = g_tab[dev][L];
    if (e.tuned)
      fprintf(f, "%u %u %u %u %.4f %.4f\n", L, e.t.sort_tile_log, e.t.sort_fmax, e.t.exp_fmax, e.sort_ms, e.exp_ms);
  }
  return fclose(f) == 0;
}

// Best of `reps` timed runs of fn() after an untimed copy of the input.
template <typename Fn>
float time_best(hipStream_t st, hipEvent_t e0, hipEvent_t e1, uint64_t* dst, const uint64_t* src, uint64_t n,
                int reps, Fn fn) {
  float best = 1e30f;
  for (int r = 0; r < reps; ++r) {
    (void)hipMemcpyAsync(dst, src, n * 8, hipMemcpyDeviceToDevice, st);
    (void)hipEventRecord(e0, st);
    fn();
    (void)hipEventRecord(e1, st);
    if (hipEventSynchronize(e1) != hipSuccess) return -1.0f;
    float ms = 0;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.0f;
    if (ms < best) best = ms;
  }
  return best;
}

int tune(uint64_t n_max, hipStream_t st, int dev) {
  uint32_t top = ilog2_ceil(n_max < 2 ? 2 : n_max);
  if (top > kTuneMaxLog) top = kTuneMaxLog;
  if (top < kTuneMinLog) return BOLT_OK;  // nothing long enough to tune
  const uint64_t nbig = 1ull << top;
  uint64_t *src = nullptr, *a = nullptr, *b = nullptr;
  if (hipMalloc((void**)&src, nbig * 8) != hipSuccess) return BOLT_ENOMEM;
  if (hipMalloc((void**)&a, nbig * 8) != hipSuccess) {
    (void)hipFree(src);
    return BOLT_ENOMEM;
  }
  if (hipMalloc((void**)&b, nbig * 8) != hipSuccess) {
    (void)hipFree(src);
    (void)hipFree(a);
    return BOLT_ENOMEM;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  int rc = BOLT_OK;
  for (uint32_t L = kTuneMinLog; L <= top && rc == BOLT_OK; ++L) {
    const uint64_t n = 1ull << L;
    const int reps = L >= 24 ? 2 : 3;
    Entry best;
    // sort: tile 2^11..2^13, 1..kSortFMax strides per global pass
    hipLaunchKernelGGL(k_tune_fill, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, st, src, n, 0u);
    float bs = 1e30f;
    for (uint32_t tl = 11; tl <= 13; ++tl)
      for (uint32_t f = 1; f <= kSortFMax; ++f) {
        const float ms = time_best(st, e0, e1, a, src, n, reps, [&] { launch_bitonic_sort_with(a, n, st, tl, f); });
        if (ms < 0) rc = BOLT_EHIP;
        if (ms >= 0 && ms < bs) {
          bs = ms;
          best.t.sort_tile_log = tl;
          best.t.sort_fmax = f;
        }
      }
    // expansion: 1..kExpFMax stages per global pass
    hipLaunchKernelGGL(k_tune_fill, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, st, src, n, 1u);
    float be = 1e30f;
    for (uint32_t f = 1; f <= kExpFMax; ++f) {
      const float ms = time_best(st, e0, e1, a, src, n, reps, [&] { (void)launch_expand_with(a, b, n, st, f); });
      if (ms < 0) rc = BOLT_EHIP;
      if (ms >= 0 && ms < be) {
        be = ms;
        best.t.exp_fmax = f;
      }
    }
    best.sort_ms = bs;
    best.exp_ms = be;
    best.tuned = true;
    if (rc == BOLT_OK) {
      std::lock_guard<std::mutex> g(g_mu);
      g_tab[dev][L] = best;
    }
  }
  (void)hipStreamSynchronize(st);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(src);
  (void)hipFree(a);
  (void)hipFree(b);
  return rc;
}

}  // namespace

namespace bolt {

NetTune net_tune(uint32_t log2n) {
  const int d = cur_dev();
  std::lock_guard<std::mutex> g(g_mu);
  return g_tab[d][log2n > kMaxLog ? kMaxLog : log2n].t;
}

}  // namespace bolt

extern "C" {

int bolt_autotune(uint64_t n_max, const char* cache_path, void* hip_stream) {
  const int dev = cur_dev();
  if (cache_path && load_cache(cache_path, dev)) return BOLT_OK;
  const int rc = tune(n_max, (hipStream_t)hip_stream, dev);
  if (rc) return rc;
  if (cache_path && !save_cache(cache_path, dev)) return BOLT_EINVAL;
  return BOLT_OK;
}

int bolt_tune_get(bolt_tune_entry* out, uint32_t cap, uint32_t* n) {
  if (!n || (cap && !out)) return BOLT_EINVAL;
  const int dev = cur_dev();
  std::lock_guard<std::mutex> g(g_mu);
  uint32_t k = 0;
  for (uint32_t L = 0; L <= kMaxLog; ++L) {
    const Entry& e = g_tab[dev][L];
    if (!e.tuned) continue;
    if (k < cap)
      out[k] = bolt_tune_entry{L, e.t.sort_tile_log, e.t.sort_fmax, e.t.exp_fmax, e.sort_ms, e.exp_ms};
    ++k;
  }
  *n = k;
  return BOLT_OK;
}

int bolt_tune_set(const bolt_tune_entry* in, uint32_t n) {
  if (n && !in) return BOLT_EINVAL;
  for (uint32_t i = 0; i < n; ++i) {
    const bolt_tune_entry& e = in[i];
    if (e.log2_n > kMaxLog || e.sort_tile_log < 11 || e.sort_tile_log > 13 || e.sort_pass_strides < 1 ||
        e.sort_pass_strides > kSortFMax || e.expand_pass_stages < 1 || e.expand_pass_stages > kExpFMax)
      return BOLT_EINVAL;
  }
  const int dev = cur_dev();
  std::lock_guard<std::mutex> g(g_mu);
  for (uint32_t i = 0; i < n; ++i) {
    Entry& t = g_tab[dev][in[i].log2_n];
    t.t = NetTune{in[i].sort_tile_log, in[i].sort_pass_strides, in[i].expand_pass_stages};
    t.sort_ms = in[i].sort_ms;
    t.exp_ms = in[i].expand_ms;
    t.tuned = true;
  }
  return BOLT_OK;
}

int bolt_tune_reset(void) {
  const int dev = cur_dev();
  std::lock_guard<std::mutex> g(g_mu);
  for (uint32_t L = 0; L <= kMaxLog; ++L) g_tab[dev][L] = Entry();
  return BOLT_OK;
}

}  // extern "C"
