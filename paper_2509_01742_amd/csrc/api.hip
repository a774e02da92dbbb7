// C ABI of the oblivious map (see include/bolt.h): parameter derivation,
// allocation of map state, argument checks, error state and readout.  All
// of the path's arithmetic runs in the kernels of k_prim / k_build /
// k_access; this file only sizes, allocates, launches and copies.
#include <math.h>
#include <string.h>
#include <sys/random.h>

#include <algorithm>
#include <mutex>
#include <new>

#include <vector>

#include "bolt_impl.h"
#include "record_dev.h"

using namespace bolt;

namespace {

constexpr uint32_t kMaxZ = 62;  // keys of a page must sit in its first 64 words
constexpr uint64_t kMaxPageBytes = 32 * 1024;  // one page is staged in a write-back wave's LDS
constexpr uint64_t kMaxSealedPage = 8 * 1024;  // four pages per fetch workgroup are opened in LDS

int derive(const bolt_params* p, Sizes* s) {
  if (!p || p->capacity < 2 || p->value_bytes == 0 || p->value_bytes % 8 || p->value_bytes > 4096) return BOLT_EINVAL;
  if (p->c == 0 || p->alpha_permille >= 1000 || p->pm_choices == 0 || p->pm_choices > 4) return BOLT_EINVAL;
  if (p->pm_keys_per_row == 0 || p->pm_row_slots == 0 || p->pm_row_slots > 32) return BOLT_EINVAL;
  if (p->observable > BOLT_OBS_DEVICE) return BOLT_EINVAL;
  if (p->capacity > (1ull << 31)) return BOLT_EINVAL;
  Sizes z{};
  z.cap = p->capacity;
  z.vs = p->value_bytes;
  z.B = (p->capacity + p->c - 1) / p->c;  // N = c (K + M)
  if (z.B < 2) return BOLT_EINVAL;
  z.K = (uint64_t)p->alpha_permille * z.B / 1000;
  z.M = z.B - z.K;
  uint32_t l1 = 0;
  while ((1ull << l1) < p->capacity) ++l1;
  uint32_t l2 = 0;
  while ((1u << l2) < l1) ++l2;
  z.lmax = p->c + l2 + 1;  // l_max of Claim 4.2 with constant 1
  // Default capacity: l_max, plus one slot when the largest batch fills at
  // least 1/64 of the bins in one placement round (B <= 64 * 8192).  Keys of
  // a round all choose on the loads at the round's start, which lifts the
  // tail of the bin loads by one over one-at-a-time placement at such fills.
  z.Z = p->bin_slots ? p->bin_slots : z.lmax + (z.B <= 64ull * kMaxBatch ? 1 : 0);
  if (z.Z == 0 || z.Z > kMaxZ) return BOLT_EINVAL;
  z.W = p->pm_row_slots;
  z.d = p->pm_choices;
  z.R = (p->capacity + p->pm_keys_per_row - 1) / p->pm_keys_per_row;
  uint64_t raw = 8 + 8 * z.Z + (uint64_t)z.vs * z.Z;
  z.page_bytes = (raw + 127) / 128 * 128;
  if (z.page_bytes > kMaxPageBytes) return BOLT_EINVAL;
  double a = (double)p->alpha_permille / 1000.0;
  double x = (1.0 + a) * (double)z.M / 2.0 + (double)z.lmax * sqrt((double)z.M * log((double)p->capacity));
  z.stash_bound = (uint64_t)ceil(x);
  // Claim 4.3 with constant 1: items the K HBM bins may hold
  z.hbm_bound = (uint64_t)ceil((double)z.K * (double)p->c +
                               (double)z.lmax * sqrt((double)z.K * log((double)p->capacity)));
  // the value pool: stash entries, plus the HBM bins' items in a decomposed store
  z.P = z.stash_bound + kMaxBatch + ((p->flags & BOLT_F_DECOMPOSED) ? z.hbm_bound : 0);
  z.BZ = z.B * z.Z;
  z.PW = (z.P + 63) / 64;
  if (z.BZ >= (1ull << 32) || z.P >= (1ull << 32)) return BOLT_EINVAL;
  // the build's P2C and position-map rounds are numbered in 16 bits
  const uint64_t rs = (z.B + 15) / 16, rsm = (z.R + 15) / 16;
  if ((z.cap + rs - 1) / rs > 0xFFFF || (z.cap + rsm - 1) / rsm > 0xFFFF) return BOLT_EINVAL;
  *s = z;
  return BOLT_OK;
}

uint64_t scratch_bytes(const Sizes& s) {
  const uint64_t Q = kMaxBatch;
  return Q * 4 * 13 + Q * s.vs + Q * 8 + 3 * Q * 4 + 2 * Q * s.page_bytes + 2 * Q * s.vs + 2 * Q + Q * 24 + 256 * 4 +
         2 * (2 * Q * s.page_bytes + 2 * Q * 4);  // two outbox halves + the page each of their slots sends
}

uint64_t device_bytes(const bolt_params* p, const Sizes& s) {
  uint64_t b = sizeof(Ctl);
  const bool decomp = (p->flags & BOLT_F_DECOMPOSED) != 0;
  if (!decomp) b += s.K * s.page_bytes;                       // HBM bins as pages
  else b += s.P * 4 + 3ull * kMaxBatch * (2 * s.Z * 4 + 1);  // the free-address ring, staged frees
  if (p->observable == BOLT_OBS_DEVICE) b += s.M * (s.page_bytes + ((p->flags & BOLT_F_SEAL) ? 16 : 0));
  if (p->flags & BOLT_F_SEAL) b += s.M * 8;  // write counts
  b += s.B * 8;                      // load, and the loads placement starts from
  b += s.R * s.W * 16 + s.R * 4;     // position map
  b += s.P * (8 + s.vs + 4 + 4) + s.PW * 8;  // stash pool + bitmap
  b += s.B * 4 + s.B * 2 * s.Z * 4;  // reverse index
  b += s.B * 16;                     // claim + rmask
  b += s.M * 8;                      // last rebuild of each observable page
  b += scratch_bytes(s);
  if (p->flags & BOLT_F_TRACE) b += p->trace_words * 4;
  return b;
}

template <typename T>
int dalloc(bolt_map* m, T** ptr, uint64_t bytes) {
  void* v = nullptr;
  if (hipMalloc(&v, bytes ? bytes : 8) != hipSuccess) return BOLT_ENOMEM;
  m->allocs.push_back(v);
  *ptr = static_cast<T*>(v);
  return BOLT_OK;
}

void free_all(bolt_map* m) {
  for (void* v : m->allocs) (void)hipFree(v);
  m->allocs.clear();
  if (m->obs_host) (void)hipHostFree(m->obs_host);
  m->obs_host = nullptr;
  for (hipGraphExec_t& g : m->gexec) {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
  if (m->side) (void)hipStreamDestroy(m->side);
  if (m->ev_fork) (void)hipEventDestroy(m->ev_fork);
  if (m->ev_join) (void)hipEventDestroy(m->ev_join);
  m->side = nullptr;
  m->ev_fork = m->ev_join = nullptr;
}

// Sends the last batch's pages to the store and waits for the map's stream.
int sync_map(bolt_map* m) {
  if (flush_ship(m, m->last_stream)) return BOLT_EHIP;
  if (hipStreamSynchronize(m->last_stream) != hipSuccess) return BOLT_EHIP;
  return BOLT_OK;
}

int map_check(bolt_map* m) {
  if (!m) return BOLT_EINVAL;
  if (m->poisoned) return BOLT_ESTATE;
  return BOLT_OK;
}

int err_code(uint32_t bits) {
  if (bits & kErrTamper) return BOLT_ETAMPER;
  if (bits & kErrBroken) return BOLT_EOVERFLOW;  // never expected: reported as a capacity failure
  if (bits & kErrOverflow) return BOLT_EOVERFLOW;
  if (bits & kErrDup) return BOLT_EDUPKEY;
  if (bits & kErrFull) return BOLT_EFULL;
  return BOLT_OK;
}

int sync_and_read(bolt_map* m, Ctl* host) {
  if (hipSetDevice(m->device) != hipSuccess) return BOLT_EHIP;
  if (sync_map(m)) return BOLT_EHIP;
  if (hipMemcpy(host, m->ctl, sizeof(Ctl), hipMemcpyDeviceToHost) != hipSuccess) return BOLT_EHIP;
  uint32_t bits = host->err & ~kErrTrace;
  if (bits && !m->poisoned) {
    m->poisoned = true;
    m->sticky = err_code(bits);
  }
  return BOLT_OK;
}

__global__ void k_fill_u8(uint8_t* p, uint64_t n, uint8_t v) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

extern "C" {

void bolt_params_default(bolt_params* p, uint64_t capacity, uint32_t value_bytes) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->capacity = capacity;
  p->value_bytes = value_bytes;
  p->c = 8;
  p->alpha_permille = 200;
  p->bin_slots = 0;
  p->pm_choices = 4;
  p->pm_keys_per_row = 16;
  p->pm_row_slots = 32;
  p->observable = BOLT_OBS_HOST_PINNED;
  p->flags = 0;
  p->trace_words = 1ull << 22;
}

int bolt_sizes_of(const bolt_params* p, bolt_sizes* out) {
  Sizes s;
  int rc = derive(p, &s);
  if (rc) return rc;
  if (out) {
    out->B = s.B;
    out->K = s.K;
    out->M = s.M;
    out->Z = s.Z;
    out->page_bytes = s.page_bytes;
    out->pm_rows = s.R;
    out->stash_bound = s.stash_bound;
    out->stash_pool = s.P;
    out->lmax = s.lmax;
    out->hbm_bound = s.hbm_bound;
  }
  return BOLT_OK;
}

int bolt_footprint(const bolt_params* p, uint64_t* hbm_bytes, uint64_t* obs_bytes) {
  Sizes s;
  int rc = derive(p, &s);
  if (rc) return rc;
  if (hbm_bytes) *hbm_bytes = device_bytes(p, s);
  if (obs_bytes) *obs_bytes = s.M * (s.page_bytes + ((p->flags & BOLT_F_SEAL) ? 16 : 0));
  return BOLT_OK;
}

int bolt_create(const bolt_params* p, void* hip_stream, bolt_map** out) {
  if (!out) return BOLT_EINVAL;
  *out = nullptr;
  Sizes s;
  int rc = derive(p, &s);
  if (rc) return rc;
  if ((p->flags & BOLT_F_TRACE) && p->trace_words == 0) return BOLT_EINVAL;
  if ((p->flags & BOLT_F_GRAPHS) && (p->flags & BOLT_F_TIMING)) return BOLT_EINVAL;
  // a fixed key would repeat the sealed store's key streams across maps
  if ((p->flags & BOLT_F_SEAL) && (p->flags & BOLT_F_FIXED_KEY) && !(p->flags & BOLT_F_SEAL_KEY_REUSE))
    return BOLT_EINVAL;
  if ((p->flags & BOLT_F_SEAL) && s.page_bytes > kMaxSealedPage) return BOLT_EINVAL;
  bolt_map* m = new (std::nothrow) bolt_map();
  if (!m) return BOLT_ENOMEM;
  m->p = *p;
  m->s = s;
  if (hipGetDevice(&m->device) != hipSuccess) {
    delete m;
    return BOLT_EHIP;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  m->last_stream = st;
  if (!(p->flags & BOLT_F_FIXED_KEY)) {
    size_t got = 0;
    while (got < 32) {
      ssize_t r = getrandom(m->p.key + got, 32 - got, 0);
      if (r <= 0) {
        delete m;
        return BOLT_EINVAL;
      }
      got += (size_t)r;
    }
  }
  const uint64_t Q = kMaxBatch;
  rc = BOLT_OK;
  rc = rc ? rc : dalloc(m, &m->ctl, sizeof(Ctl));
  if (p->flags & BOLT_F_DECOMPOSED)  // no HBM pages: the ring of the value pool instead
    rc = rc ? rc : dalloc(m, &m->ring, s.P * 4);
  else
    rc = rc ? rc : dalloc(m, &m->hbm, s.K * s.page_bytes);
  rc = rc ? rc : dalloc(m, &m->load, s.B * 4);
  rc = rc ? rc : dalloc(m, &m->load0, s.B * 4);
  rc = rc ? rc : dalloc(m, &m->pm_key, s.R * s.W * 8);
  rc = rc ? rc : dalloc(m, &m->pm_pair, s.R * s.W * 8);
  rc = rc ? rc : dalloc(m, &m->pm_mask, s.R * 4);
  rc = rc ? rc : dalloc(m, &m->st_key, s.P * 8);
  rc = rc ? rc : dalloc(m, &m->st_val, s.P * s.vs);
  rc = rc ? rc : dalloc(m, &m->st_dest, s.P * 4);
  rc = rc ? rc : dalloc(m, &m->st_dead, s.P * 4);
  rc = rc ? rc : dalloc(m, &m->st_used, s.PW * 8);
  rc = rc ? rc : dalloc(m, &m->rev_cnt, s.B * 4);
  rc = rc ? rc : dalloc(m, &m->rev_idx, s.B * 2 * s.Z * 4);
  rc = rc ? rc : dalloc(m, &m->claim, s.B * 8);
  rc = rc ? rc : dalloc(m, &m->rmask, s.B * 8);
  BatchScratch& b = m->bs;
  rc = rc ? rc : dalloc(m, &b.leader, Q * 4);
  rc = rc ? rc : dalloc(m, &b.prevw, Q * 4);
  rc = rc ? rc : dalloc(m, &b.lastw, Q * 4);
  rc = rc ? rc : dalloc(m, &b.hit, Q * 4);
  rc = rc ? rc : dalloc(m, &b.hrow, Q * 4);
  rc = rc ? rc : dalloc(m, &b.hslot, Q * 4);
  rc = rc ? rc : dalloc(m, &b.found, Q * 4);
  rc = rc ? rc : dalloc(m, &b.fval, Q * s.vs);
  rc = rc ? rc : dalloc(m, &b.rpair, Q * 8);
  rc = rc ? rc : dalloc(m, &b.cand_bin, 3 * Q * 4);
  rc = rc ? rc : dalloc(m, &b.stage, 2 * Q * s.page_bytes);
  rc = rc ? rc : dalloc(m, &b.outbox, 2 * 2 * Q * s.page_bytes);
  rc = rc ? rc : dalloc(m, &b.ship_page, 2 * 2 * Q * 4);
  rc = rc ? rc : dalloc(m, &m->wslot, s.M * 8);
  rc = rc ? rc : dalloc(m, &b.fin, Q * 4);
  rc = rc ? rc : dalloc(m, &b.chosen, Q * 4);
  rc = rc ? rc : dalloc(m, &b.rowsel, Q * 4);
  rc = rc ? rc : dalloc(m, &b.freed, 256 * 4);
  rc = rc ? rc : dalloc(m, &b.fpair, Q * 8);
  rc = rc ? rc : dalloc(m, &b.rows, Q * 16);
  if (p->flags & BOLT_F_DECOMPOSED) {
    rc = rc ? rc : dalloc(m, &b.rfree, 3 * Q * 2 * s.Z * 4);
    rc = rc ? rc : dalloc(m, &b.rfree_n, 3 * Q);
  }
  rc = rc ? rc : dalloc(m, &m->get_ops, Q);
  rc = rc ? rc : dalloc(m, &m->put_ops, Q);
  rc = rc ? rc : dalloc(m, &m->discard, 2 * Q * s.vs);
  if (!rc && (p->flags & BOLT_F_TRACE)) {
    m->tlog_cap = p->trace_words;
    rc = dalloc(m, &m->tlog, m->tlog_cap * 4);
  }
  if (!rc && (p->flags & BOLT_F_SEAL)) rc = dalloc(m, &m->pver, s.M * 8);
  if (!rc && (p->flags & BOLT_F_SEAL_CMDS)) {
    rc = dalloc(m, &m->sc_ops, Q);
    rc = rc ? rc : dalloc(m, &m->sc_keys, Q * 8);
    rc = rc ? rc : dalloc(m, &m->sc_vin, Q * s.vs);
    rc = rc ? rc : dalloc(m, &m->sc_vout, Q * s.vs);
    rc = rc ? rc : dalloc(m, &m->sc_st, Q);
  }
  if (!rc) {
    const uint64_t ob = s.M * s.page_bytes + ((p->flags & BOLT_F_SEAL) ? s.M * 16 : 0);  // pages, then tags
    if (p->observable == BOLT_OBS_DEVICE) {
      rc = dalloc(m, &m->obs, ob);
    } else {
      void* h = nullptr;
      if (hipHostMalloc(&h, ob ? ob : 8, hipHostMallocMapped) != hipSuccess) {
        rc = BOLT_ENOMEM;
      } else {
        m->obs_host = static_cast<uint8_t*>(h);
        void* d = nullptr;
        if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) rc = BOLT_EHIP;
        m->obs = static_cast<uint8_t*>(d);
      }
    }
  }
  if (!rc && (p->flags & BOLT_F_SEAL)) m->tags = m->obs + s.M * s.page_bytes;
  if (rc) {
    free_all(m);
    delete m;
    return rc;
  }
  if (hipStreamCreateWithFlags(&m->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&m->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&m->ev_join, hipEventDisableTiming) != hipSuccess) {
    free_all(m);
    delete m;
    return BOLT_EHIP;
  }
  if (p->flags & BOLT_F_TIMING) {
    m->timer = new (std::nothrow) KernelTimer();
    if (!m->timer) {
      free_all(m);
      delete m;
      return BOLT_ENOMEM;
    }
  }
  launch_map_init(m, st);
  if (p->flags & BOLT_F_SEAL_CMDS)  // the session key goes to device memory (the pageable copy completes here)
    (void)hipMemcpyAsync(m->ctl->ckey, p->session_key, 32, hipMemcpyHostToDevice, st);
  (void)hipMemsetAsync(m->bs.freed, 0, 256 * 4, st);
  (void)hipMemsetAsync(m->wslot, 0, s.M * 8, st);  // epoch 0: no page rebuilt yet

  hipLaunchKernelGGL(k_fill_u8, dim3((uint32_t)((Q + 255) / 256)), dim3(256), 0, st, m->get_ops, Q, (uint8_t)0);
  hipLaunchKernelGGL(k_fill_u8, dim3((uint32_t)((Q + 255) / 256)), dim3(256), 0, st, m->put_ops, Q, (uint8_t)1);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
    free_all(m);
    delete m;
    return BOLT_EHIP;
  }
  *out = m;
  return BOLT_OK;
}

int bolt_build(bolt_map* m, const uint64_t* d_keys, const void* d_vals, uint64_t n, void* hip_stream) {
  int rc = map_check(m);
  if (rc) return rc;
  if (m->built || n > m->s.cap) return BOLT_EINVAL;
  if (n && (!d_keys || !d_vals)) return BOLT_EINVAL;
  if (((uintptr_t)d_keys | (uintptr_t)d_vals) & 7) return BOLT_EINVAL;
  hipStream_t st = (hipStream_t)hip_stream;
  m->last_stream = st;
  if (hipSetDevice(m->device) != hipSuccess) return BOLT_EHIP;
  rc = run_build(m, d_keys, d_vals, n, st);
  if (rc) return rc;
  m->built = true;
  return BOLT_OK;
}

int bolt_build_many(bolt_map* const* maps, const uint64_t* const* d_keys, const void* const* d_vals,
                    const uint64_t* n, uint32_t count, void* hip_stream) {
  if (count == 0) return BOLT_OK;
  if (!maps || !d_keys || !d_vals || !n) return BOLT_EINVAL;
  for (uint32_t i = 0; i < count; ++i) {
    bolt_map* m = maps[i];
    int rc = map_check(m);
    if (rc) return rc;
    if (m->built || n[i] > m->s.cap) return BOLT_EINVAL;
    if (m->device != maps[0]->device) return BOLT_EINVAL;
    if (n[i] && (!d_keys[i] || !d_vals[i])) return BOLT_EINVAL;
    if (((uintptr_t)d_keys[i] | (uintptr_t)d_vals[i]) & 7) return BOLT_EINVAL;
    for (uint32_t j = 0; j < i; ++j)
      if (maps[j] == m) return BOLT_EINVAL;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  if (hipSetDevice(maps[0]->device) != hipSuccess) return BOLT_EHIP;
  int rc = count == 1 ? run_build(maps[0], d_keys[0], d_vals[0], n[0], st)
                      : run_build_many(maps, d_keys, d_vals, n, count, st);
  if (rc) return rc;
  for (uint32_t i = 0; i < count; ++i) {
    maps[i]->last_stream = st;
    maps[i]->built = true;
  }
  return BOLT_OK;
}

int bolt_access_batch(bolt_map* m, const uint8_t* d_ops, const uint64_t* d_keys, const void* d_vals_in,
                      void* d_vals_out, uint8_t* d_status, uint32_t q, void* hip_stream) {
  int rc = map_check(m);
  if (rc) return rc;
  if (!m->built || q > kMaxBatch) return BOLT_EINVAL;
  if (q == 0) return BOLT_OK;
  if (!d_ops || !d_keys || !d_vals_in || !d_vals_out || !d_status) return BOLT_EINVAL;
  if (((uintptr_t)d_keys | (uintptr_t)d_vals_in | (uintptr_t)d_vals_out) & 7) return BOLT_EINVAL;
  hipStream_t st = (hipStream_t)hip_stream;
  m->last_stream = st;
  if (hipSetDevice(m->device) != hipSuccess) return BOLT_EHIP;
  return run_access(m, d_ops, d_keys, d_vals_in, d_vals_out, d_status, q, st);
}

int bolt_access_many(bolt_map* const* maps, const bolt_batch* batches, uint32_t count, void* hip_stream) {
  return access_many(maps, batches, count, hip_stream, false);
}

}  // extern "C"

int bolt::access_many(bolt_map* const* maps, const bolt_batch* batches, uint32_t count, void* hip_stream,
                      bool defer_pages) {
  if (count == 0) return BOLT_OK;
  if (!maps || !batches) return BOLT_EINVAL;
  std::vector<bolt_map*> live;
  std::vector<bolt_batch> work;
  live.reserve(count);
  work.reserve(count);
  for (uint32_t i = 0; i < count; ++i) {
    bolt_map* m = maps[i];
    int rc = map_check(m);
    if (rc) return rc;
    const bolt_batch& b = batches[i];
    if (!m->built || b.q > kMaxBatch) return BOLT_EINVAL;
    if (m->device != maps[0]->device) return BOLT_EINVAL;
    for (uint32_t j = 0; j < i; ++j)
      if (maps[j] == m) return BOLT_EINVAL;  // one batch per map and call
    if (b.q == 0) continue;
    if (!b.d_ops || !b.d_keys || !b.d_vals_in || !b.d_vals_out || !b.d_status) return BOLT_EINVAL;
    if (((uintptr_t)b.d_keys | (uintptr_t)b.d_vals_in | (uintptr_t)b.d_vals_out) & 7) return BOLT_EINVAL;
    live.push_back(m);
    work.push_back(b);
  }
  if (live.empty()) return BOLT_OK;
  hipStream_t st = (hipStream_t)hip_stream;
  if (hipSetDevice(live[0]->device) != hipSuccess) return BOLT_EHIP;
  for (bolt_map* m : live) m->last_stream = st;
  if (live.size() == 1)
    return run_access(live[0], work[0].d_ops, work[0].d_keys, work[0].d_vals_in, work[0].d_vals_out,
                      work[0].d_status, work[0].q, st);
  return run_access_many(live.data(), work.data(), (uint32_t)live.size(), st, defer_pages);
}

extern "C" {

int bolt_access_sealed(bolt_map* m, const void* d_req, uint32_t q, void* d_resp, void* hip_stream) {
  int rc = map_check(m);
  if (rc) return rc;
  if (!m->built || !(m->p.flags & BOLT_F_SEAL_CMDS) || q == 0 || q > kMaxBatch || !d_req || !d_resp)
    return BOLT_EINVAL;
  if (((uintptr_t)d_req | (uintptr_t)d_resp) & 7) return BOLT_EINVAL;
  hipStream_t st = (hipStream_t)hip_stream;
  m->last_stream = st;
  if (hipSetDevice(m->device) != hipSuccess) return BOLT_EHIP;
  launch_rec_open(m, d_req, q, nullptr, 1, m->sc_ops, m->sc_keys, m->sc_vin, st);
  rc = run_access(m, m->sc_ops, m->sc_keys, m->sc_vin, m->sc_vout, m->sc_st, q, st);
  if (rc) return rc;
  launch_rec_seal(m, d_resp, q, nullptr, 1, m->sc_st, m->sc_vout, st);
  return hipGetLastError() == hipSuccess ? BOLT_OK : BOLT_EHIP;
}

int bolt_get_batch(bolt_map* m, const uint64_t* d_keys, uint32_t q, void* d_vals_out, uint8_t* d_found,
                   void* hip_stream) {
  int rc = map_check(m);
  if (rc) return rc;
  if (!m->built || q > kMaxBatch) return BOLT_EINVAL;
  if (q == 0) return BOLT_OK;
  if (!d_keys || !d_vals_out || !d_found) return BOLT_EINVAL;
  if (((uintptr_t)d_keys | (uintptr_t)d_vals_out) & 7) return BOLT_EINVAL;
  hipStream_t st = (hipStream_t)hip_stream;
  m->last_stream = st;
  if (hipSetDevice(m->device) != hipSuccess) return BOLT_EHIP;
  // GET status is 1 for a present key and 0 otherwise: exactly d_found.
  return run_access(m, m->get_ops, d_keys, m->discard, d_vals_out, d_found, q, st);
}

int bolt_put_batch(bolt_map* m, const uint64_t* d_keys, const void* d_vals, uint32_t q, uint8_t* d_status,
                   void* hip_stream) {
  int rc = map_check(m);
  if (rc) return rc;
  if (!m->built || q > kMaxBatch) return BOLT_EINVAL;
  if (q == 0) return BOLT_OK;
  if (!d_keys || !d_vals || !d_status) return BOLT_EINVAL;
  if (((uintptr_t)d_keys | (uintptr_t)d_vals) & 7) return BOLT_EINVAL;
  hipStream_t st = (hipStream_t)hip_stream;
  m->last_stream = st;
  if (hipSetDevice(m->device) != hipSuccess) return BOLT_EHIP;
  return run_access(m, m->put_ops, d_keys, d_vals, m->discard + (uint64_t)kMaxBatch * m->s.vs, d_status, q, st);
}

int bolt_destroy(bolt_map* m) {
  if (!m) return BOLT_OK;
  (void)hipSetDevice(m->device);
  (void)hipStreamSynchronize(m->last_stream);  // pages still to be sent die with the map
  if (m->side) (void)hipStreamSynchronize(m->side);
  delete m->timer;
  free_all(m);
  delete m;
  return BOLT_OK;
}

int bolt_flush(bolt_map* m, void* hip_stream) {
  if (!m) return BOLT_EINVAL;
  hipStream_t st = (hipStream_t)hip_stream;
  if (hipSetDevice(m->device) != hipSuccess) return BOLT_EHIP;
  m->last_stream = st;
  return flush_ship(m, st);
}

int bolt_status(bolt_map* m) {
  if (!m) return BOLT_EINVAL;
  Ctl c;
  int rc = sync_and_read(m, &c);
  if (rc) return rc;
  return m->poisoned ? m->sticky : BOLT_OK;
}

int bolt_map_sizes(const bolt_map* m, bolt_sizes* out) {
  if (!m || !out) return BOLT_EINVAL;
  return bolt_sizes_of(&m->p, out);
}

int bolt_get_stats(bolt_map* m, bolt_stats* out) {
  if (!m || !out) return BOLT_EINVAL;
  Ctl c;
  int rc = sync_and_read(m, &c);
  if (rc) return rc;
  const Sizes& s = m->s;
  memset(out, 0, sizeof(*out));
  out->live = c.live;
  out->steps = c.steps;
  out->batches = m->batches;
  out->stash_live = c.stash_live;
  out->stash_highwater = c.stash_hw;
  std::vector<uint32_t> ld(s.B);
  if (hipMemcpy(ld.data(), m->load, s.B * 4, hipMemcpyDeviceToHost) != hipSuccess) return BOLT_EHIP;
  out->max_load = *std::max_element(ld.begin(), ld.end());
  std::vector<uint32_t> mk(s.R);
  if (hipMemcpy(mk.data(), m->pm_mask, s.R * 4, hipMemcpyDeviceToHost) != hipSuccess) return BOLT_EHIP;
  uint32_t mr = 0;
  for (uint32_t v : mk) mr = std::max(mr, (uint32_t)__builtin_popcount(v));
  out->max_row = mr;
  out->load_highwater = c.load_hw;
  out->hbm_load = c.hbm_load;
  out->hbm_load_highwater = c.hbm_hw;
  return BOLT_OK;
}

int bolt_trace_read(bolt_map* m, bolt_trace_rec* host_recs, uint64_t cap, uint64_t* n) {
  if (!m || !n) return BOLT_EINVAL;
  if (!m->tlog) return BOLT_EINVAL;
  Ctl c;
  int rc = sync_and_read(m, &c);
  if (rc) return rc;
  std::vector<uint32_t> log(m->tlog_used);
  if (m->tlog_used &&
      hipMemcpy(log.data(), m->tlog, m->tlog_used * 4, hipMemcpyDeviceToHost) != hipSuccess)
    return BOLT_EHIP;
  uint64_t k = 0;
  std::vector<uint32_t> w;
  for (const TraceSeg& g : m->segs) {
    for (uint64_t x = 0; x < g.reads; ++x) {
      uint32_t v = log[g.offset + x];
      if (v == kNone) continue;
      if (k < cap && host_recs) host_recs[k] = bolt_trace_rec{g.batch, 0, v};
      ++k;
    }
    w.clear();
    for (uint64_t x = 0; x < g.writes; ++x) {
      uint32_t v = log[g.offset + g.reads + x];
      if (v != kNone) w.push_back(v);
    }
    std::sort(w.begin(), w.end());
    for (uint32_t v : w) {
      if (k < cap && host_recs) host_recs[k] = bolt_trace_rec{g.batch, 1, v};
      ++k;
    }
  }
  *n = k;
  return m->tlog_lost ? BOLT_EFULL : BOLT_OK;
}

int bolt_trace_clear(bolt_map* m) {
  if (!m || !m->tlog) return BOLT_EINVAL;
  Ctl c;
  int rc = sync_and_read(m, &c);
  if (rc) return rc;
  m->segs.clear();
  m->tlog_used = 0;
  m->tlog_lost = false;
  return BOLT_OK;
}

int bolt_observable_snapshot(bolt_map* m, void* host_buf, uint64_t cap) {
  if (!m || !host_buf) return BOLT_EINVAL;
  const uint64_t bytes = m->s.M * m->s.page_bytes;
  if (cap < bytes) return BOLT_EINVAL;
  Ctl c;
  int rc = sync_and_read(m, &c);
  if (rc) return rc;
  if (m->obs_host) {
    memcpy(host_buf, m->obs_host, bytes);
    return BOLT_OK;
  }
  return hipMemcpy(host_buf, m->obs, bytes, hipMemcpyDeviceToHost) == hipSuccess ? BOLT_OK : BOLT_EHIP;
}

int bolt_tags_snapshot(bolt_map* m, void* host_buf, uint64_t cap) {
  if (!m || !host_buf || !m->tags) return BOLT_EINVAL;
  const uint64_t bytes = m->s.M * 16;
  if (cap < bytes) return BOLT_EINVAL;
  Ctl c;
  int rc = sync_and_read(m, &c);
  if (rc) return rc;
  if (m->obs_host) {
    memcpy(host_buf, m->obs_host + m->s.M * m->s.page_bytes, bytes);
    return BOLT_OK;
  }
  return hipMemcpy(host_buf, m->tags, bytes, hipMemcpyDeviceToHost) == hipSuccess ? BOLT_OK : BOLT_EHIP;
}

int bolt_versions_snapshot(bolt_map* m, uint64_t* host_buf, uint64_t cap) {
  if (!m || !host_buf || !m->pver || cap < m->s.M) return BOLT_EINVAL;
  Ctl c;
  int rc = sync_and_read(m, &c);
  if (rc) return rc;
  return hipMemcpy(host_buf, m->pver, m->s.M * 8, hipMemcpyDeviceToHost) == hipSuccess ? BOLT_OK : BOLT_EHIP;
}

int bolt_observable_raw(bolt_map* m, uint64_t page, void* host_buf, int write) {
  if (!m || !host_buf || !m->tags || page >= m->s.M) return BOLT_EINVAL;
  Ctl c;
  int rc = sync_and_read(m, &c);
  if (rc) return rc;
  const uint64_t pb = m->s.page_bytes;
  uint8_t* buf = static_cast<uint8_t*>(host_buf);
  uint8_t* pg = m->obs + page * pb;
  uint8_t* tg = m->tags + page * 16;
  // A page changed from the host is read back from the store, not from the
  // outbox of the last batch's rebuilt pages.
  if (write) m->ov_off = true;
  if (m->obs_host) {  // pinned memory: the host's own view
    pg = m->obs_host + page * pb;
    tg = m->obs_host + m->s.M * pb + page * 16;
    if (write) {
      memcpy(pg, buf, pb);
      memcpy(tg, buf + pb, 16);
    } else {
      memcpy(buf, pg, pb);
      memcpy(buf + pb, tg, 16);
    }
    return BOLT_OK;
  }
  const hipMemcpyKind k = write ? hipMemcpyHostToDevice : hipMemcpyDeviceToHost;
  if (hipMemcpy(write ? (void*)pg : buf, write ? (const void*)buf : pg, pb, k) != hipSuccess) return BOLT_EHIP;
  if (hipMemcpy(write ? (void*)tg : buf + pb, write ? (const void*)(buf + pb) : tg, 16, k) != hipSuccess)
    return BOLT_EHIP;
  return BOLT_OK;
}

int bolt_hbm_snapshot(bolt_map* m, void* host_buf, uint64_t cap) {
  if (!m || (!host_buf && m->s.K)) return BOLT_EINVAL;
  const uint64_t bytes = m->s.K * m->s.page_bytes;
  if (cap < bytes) return BOLT_EINVAL;
  Ctl c;
  int rc = sync_and_read(m, &c);
  if (rc) return rc;
  if (!bytes) return BOLT_OK;
  if (!m->hbm) {  // decomposed store: no HBM pages, every bin reads as empty
    memset(host_buf, 0, bytes);
    return BOLT_OK;
  }
  return hipMemcpy(host_buf, m->hbm, bytes, hipMemcpyDeviceToHost) == hipSuccess ? BOLT_OK : BOLT_EHIP;
}

int bolt_loads_snapshot(bolt_map* m, uint32_t* host_buf, uint64_t cap) {
  if (!m || !host_buf || cap < m->s.B * 4) return BOLT_EINVAL;
  Ctl c;
  int rc = sync_and_read(m, &c);
  if (rc) return rc;
  return hipMemcpy(host_buf, m->load, m->s.B * 4, hipMemcpyDeviceToHost) == hipSuccess ? BOLT_OK : BOLT_EHIP;
}

int bolt_stash_snapshot(bolt_map* m, uint64_t* host_keys, uint32_t* host_bins, void* host_vals, uint64_t cap,
                        uint64_t* n) {
  if (!m || !n) return BOLT_EINVAL;
  Ctl c;
  int rc = sync_and_read(m, &c);
  if (rc) return rc;
  const Sizes& s = m->s;
  std::vector<uint64_t> used(s.PW);
  std::vector<uint32_t> dest(s.P);
  std::vector<uint64_t> key(s.P);
  std::vector<uint8_t> val(s.P * s.vs);
  if (hipMemcpy(used.data(), m->st_used, s.PW * 8, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(dest.data(), m->st_dest, s.P * 4, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(key.data(), m->st_key, s.P * 8, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(val.data(), m->st_val, s.P * s.vs, hipMemcpyDeviceToHost) != hipSuccess)
    return BOLT_EHIP;
  std::vector<uint8_t> is_free(s.P, 0);
  if (m->ring) {  // decomposed store: the free entries are those in the ring's free range, each once
    std::vector<uint32_t> ring(s.P);
    if (hipMemcpy(ring.data(), m->ring, s.P * 4, hipMemcpyDeviceToHost) != hipSuccess) return BOLT_EHIP;
    if (c.ring_tail < c.ring_head || c.ring_tail - c.ring_head > s.P) return BOLT_ESTATE;
    for (uint64_t j = c.ring_head; j < c.ring_tail; ++j) {
      const uint32_t e = ring[j % s.P];
      if (e >= s.P || is_free[e]) return BOLT_ESTATE;  // the ring lost its shape (a library bug)
      is_free[e] = 1;
    }
  } else {
    for (uint64_t e = 0; e < s.P; ++e) is_free[e] = !((used[e >> 6] >> (e & 63)) & 1);
  }
  uint64_t k = 0;
  for (uint64_t e = 0; e < s.P; ++e) {
    if (is_free[e]) continue;
    if (k < cap) {
      if (host_keys) host_keys[k] = key[e];
      if (host_bins) host_bins[k] = dest[e];
      if (host_vals) memcpy(static_cast<uint8_t*>(host_vals) + k * s.vs, &val[e * s.vs], s.vs);
    }
    ++k;
  }
  *n = k;
  return BOLT_OK;
}

int bolt_pm_snapshot(bolt_map* m, uint64_t* host_rows, uint64_t* host_keys, uint32_t* host_p1, uint32_t* host_p2,
                     uint64_t cap, uint64_t* n) {
  if (!m || !n) return BOLT_EINVAL;
  Ctl c;
  int rc = sync_and_read(m, &c);
  if (rc) return rc;
  const Sizes& s = m->s;
  std::vector<uint32_t> mask(s.R);
  std::vector<uint64_t> key(s.R * s.W);
  std::vector<uint2> pr(s.R * s.W);
  if (hipMemcpy(mask.data(), m->pm_mask, s.R * 4, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(key.data(), m->pm_key, s.R * s.W * 8, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(pr.data(), m->pm_pair, s.R * s.W * 8, hipMemcpyDeviceToHost) != hipSuccess)
    return BOLT_EHIP;
  uint64_t k = 0;
  for (uint64_t r = 0; r < s.R; ++r)
    for (uint32_t j = 0; j < s.W; ++j) {
      if (!((mask[r] >> j) & 1)) continue;
      if (k < cap) {
        if (host_rows) host_rows[k] = r;
        if (host_keys) host_keys[k] = key[r * s.W + j];
        if (host_p1) host_p1[k] = pr[r * s.W + j].x;
        if (host_p2) host_p2[k] = pr[r * s.W + j].y;
      }
      ++k;
    }
  *n = k;
  return BOLT_OK;
}

int bolt_kernel_times(bolt_map* m, bolt_kernel_time* host_out, uint32_t cap, uint32_t* n) {
  if (!m || !n || !m->timer) return BOLT_EINVAL;
  if (hipSetDevice(m->device) != hipSuccess || sync_map(m)) return BOLT_EHIP;
  if (m->timer->collect()) return BOLT_EHIP;
  for (uint32_t i = 0; i < (uint32_t)kkCount && i < cap && host_out; ++i) {
    memset(&host_out[i], 0, sizeof(host_out[i]));
    strncpy(host_out[i].name, kKernelNames[i], sizeof(host_out[i].name) - 1);
    host_out[i].launches = m->timer->launches[i];
    host_out[i].total_ms = m->timer->total_ms[i];
  }
  *n = kkCount;
  return BOLT_OK;
}

int bolt_kernel_times_reset(bolt_map* m) {
  if (!m || !m->timer) return BOLT_EINVAL;
  if (hipSetDevice(m->device) != hipSuccess || sync_map(m)) return BOLT_EHIP;
  if (m->timer->collect()) return BOLT_EHIP;
  m->timer->reset();
  return BOLT_OK;
}

// ---- client side of sealed requests (host code) ----

static void key_words(const uint8_t* k, uint32_t w[8]) {
  for (int j = 0; j < 8; ++j)
    w[j] = (uint32_t)k[4 * j] | ((uint32_t)k[4 * j + 1] << 8) | ((uint32_t)k[4 * j + 2] << 16) |
           ((uint32_t)k[4 * j + 3] << 24);
}

static uint64_t ld64(const uint8_t* p) {
  uint64_t v;
  memcpy(&v, p, 8);
  return v;
}

static void st64(uint8_t* p, uint64_t v) { memcpy(p, &v, 8); }

int bolt_seal_requests(const uint8_t* session_key, uint64_t seq, uint32_t q, uint32_t value_bytes,
                       const uint8_t* ops, const uint64_t* keys, const void* vals, void* out_records) {
  if (!session_key || value_bytes == 0 || value_bytes % 8) return BOLT_EINVAL;
  if (q && (!ops || !keys || !vals || !out_records)) return BOLT_EINVAL;
  uint32_t key[8];
  key_words(session_key, key);
  const uint32_t vw = value_bytes / 8, words = 2 + vw;
  const uint8_t* v = static_cast<const uint8_t*>(vals);
  for (uint32_t i = 0; i < q; ++i) {
    uint8_t* rec = static_cast<uint8_t*>(out_records) + (uint64_t)i * (words + 2) * 8;
    RecStream ks{key, i, (uint32_t)seq, (uint32_t)(seq >> 32)};
    st64(rec, (uint64_t)ops[i] ^ ks.word(0));
    st64(rec + 8, keys[i] ^ ks.word(1));
    for (uint32_t w = 0; w < vw; ++w) st64(rec + 8 * (2 + w), ld64(v + ((uint64_t)i * vw + w) * 8) ^ ks.word(2 + w));
    uint32_t otk[8], tag[4];
    rec_otk(key, i, seq, otk);
    rec_tag(otk, q, words, [&](uint32_t w) { return ld64(rec + 8 * w); }, tag);
    memcpy(rec + 8 * words, tag, 16);
  }
  return BOLT_OK;
}

int bolt_open_responses(const uint8_t* session_key, uint64_t seq, uint32_t q, uint32_t value_bytes,
                        const void* records, uint8_t* status, void* vals) {
  if (!session_key || value_bytes == 0 || value_bytes % 8) return BOLT_EINVAL;
  if (q && (!records || !status || !vals)) return BOLT_EINVAL;
  uint32_t key[8];
  key_words(session_key, key);
  const uint32_t vw = value_bytes / 8, words = 1 + vw;
  uint8_t* v = static_cast<uint8_t*>(vals);
  int rc = BOLT_OK;
  for (uint32_t i = 0; i < q; ++i) {
    const uint8_t* rec = static_cast<const uint8_t*>(records) + (uint64_t)i * (words + 2) * 8;
    uint32_t otk[8], tag[4];
    rec_otk(key, i | kRespDir, seq, otk);
    rec_tag(otk, q, words, [&](uint32_t w) { return ld64(rec + 8 * w); }, tag);
    if (memcmp(tag, rec + 8 * words, 16) != 0) {
      rc = BOLT_ETAMPER;
      status[i] = 0;
      memset(v + (uint64_t)i * value_bytes, 0, value_bytes);
      continue;
    }
    RecStream ks{key, i | kRespDir, (uint32_t)seq, (uint32_t)(seq >> 32)};
    status[i] = (uint8_t)(ld64(rec) ^ ks.word(0));
    for (uint32_t w = 0; w < vw; ++w) st64(v + ((uint64_t)i * vw + w) * 8, ld64(rec + 8 * (1 + w)) ^ ks.word(1 + w));
  }
  return rc;
}

}  // extern "C"

// Scratch of the allocation-free expansion: one static array per device,
// held until the process ends.  In host code `scratch` names a host-side
// stand-in, so its device address is looked up once per device (with that
// device current) and only that address is handed to kernels.
static __device__ __align__(256) uint64_t scratch[BOLT_NOALLOC_EXPAND_MAX];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
uint64_t* g_scratch_ptr[kScratchDevices];
}  // namespace

static int noalloc_scratch(uint64_t** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kScratchDevices) return BOLT_EHIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return BOLT_EHIP;
    g_scratch_ptr[dev] = static_cast<uint64_t*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return BOLT_OK;
}

extern "C" {

int bolt_prf(const uint8_t* host_key, uint8_t domain, const uint64_t* d_x, uint64_t n, uint64_t* d_out,
             void* hip_stream) {
  if (!host_key || (n && (!d_x || !d_out))) return BOLT_EINVAL;
  if (n == 0) return BOLT_OK;
  hipStream_t st = (hipStream_t)hip_stream;
  Ctl* ctl = nullptr;
  if (hipMallocAsync((void**)&ctl, sizeof(Ctl), st) != hipSuccess) return BOLT_ENOMEM;
  launch_prf_key_setup(ctl, host_key, st);
  launch_prf_array(ctl, domain, d_x, n, d_out, st);
  (void)hipFreeAsync(ctl, st);
  return hipGetLastError() == hipSuccess ? BOLT_OK : BOLT_EHIP;
}

int bolt_sort_u64(uint64_t* d_data, uint64_t n, void* hip_stream) {
  if (!d_data || n == 0 || (n & (n - 1)) || n > (1ull << 31)) return BOLT_EINVAL;
  launch_bitonic_sort(d_data, n, (hipStream_t)hip_stream);
  return hipGetLastError() == hipSuccess ? BOLT_OK : BOLT_EHIP;
}

int bolt_expand_u64(uint64_t* d_elems, uint64_t* d_tmp, uint64_t m, void* hip_stream) {
  if (!d_elems || !d_tmp || m == 0 || m > (1ull << 32)) return BOLT_EINVAL;
  launch_expand(d_elems, d_tmp, m, (hipStream_t)hip_stream);
  return hipGetLastError() == hipSuccess ? BOLT_OK : BOLT_EHIP;
}

int bolt_expand_u64_noalloc(uint64_t* d_elems, uint64_t m, void* hip_stream) {
  if (!d_elems || m == 0) return BOLT_EINVAL;
  if (m > BOLT_NOALLOC_EXPAND_MAX) return BOLT_EINVAL;  // larger than the static scratch
  uint64_t* tmp = nullptr;
  const int rc = noalloc_scratch(&tmp);
  if (rc) return rc;
  launch_expand(d_elems, tmp, m, (hipStream_t)hip_stream);
  return hipGetLastError() == hipSuccess ? BOLT_OK : BOLT_EHIP;
}

}  // extern "C"
