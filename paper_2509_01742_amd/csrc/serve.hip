// Serving loop: many resident maps behind one request queue.
//
// The device holds every admitted map's state; the host only relays
// commands and responses (the self-hosted model of Sec. 5.1, with host
// buffers pooling commands and responses as the paper's I/O buffers do).
//
//   admission   a map opened on the server is created and built once its
//               device footprint (bolt_footprint plus its command staging)
//               fits the HBM budget; until then its requests wait.  Closing
//               a map frees its share and admits the next waiting one.
//               Creating, building and freeing maps (allocations, the
//               build's input copies, device-wide frees) run on a builder
//               thread, so the serving loop never stalls on them; maps
//               admitted together are built with one multi-map build.
//   batching    continuous: on every turn of the loop, each admitted map
//               that is idle and has queued requests takes its queue head,
//               as many whole requests as fit one batch, in FIFO order; all
//               maps taken on one turn run as one multi-map access (one
//               launch per phase for all of them) on a free stream.  Work
//               that arrives while groups run joins the next turn, on
//               another stream, so groups of different maps overlap.
//   results     a request's answers are those of its commands run in order
//               after every earlier request of its map (batches follow
//               sequential semantics), so they do not depend on what else
//               runs beside it.
//   latency     completion time minus the arrival time given at submit.
//   sealing     a map created with BOLT_F_SEAL_CMDS takes only sealed
//               requests: the host stages their command records and the
//               response records come back, so plain commands and results
//               exist only in device memory.  Its requests are numbered in
//               submission order (the order the map runs them).
#include <string.h>
#include <time.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "bolt_impl.h"

using namespace bolt;

namespace {

constexpr int32_t kPending = 1;

uint64_t now_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

struct Req {
  uint64_t ticket;
  const uint8_t* ops;
  const uint64_t* keys;
  const uint8_t* vin;
  uint8_t* vout;
  uint8_t* status;
  uint32_t q;
  uint64_t t_arr;
  const uint8_t* rec_in;  // sealed request: its command records (else null)
  uint8_t* rec_out;       // and where its response records go
};

// kQueued: admitted, waiting for the builder; kRetiring: its resources are
// being freed (then kClosed or kFailed).
enum MapState { kWaiting, kQueued, kBuilding, kResident, kRetiring, kClosed, kFailed };

// Command staging of one map: [ops Q][keys Q][vals_in Q*vs][vals_out Q*vs]
// [status Q][error word], and for a sealed map [request starts Q+1]
// [command records Q*(32+vs)][response records Q*(24+vs)].  A sealed map's
// host staging uses only the error word and the sealed part.
struct Stage {
  uint8_t* base = nullptr;
  uint64_t off_keys = 0, off_vin = 0, off_vout = 0, off_st = 0, off_err = 0, bytes = 0;
  uint64_t off_tab = 0, off_req = 0, off_resp = 0;
  void layout(uint32_t Q, uint32_t vs, bool sealed) {
    off_keys = (Q + 255) & ~255ull;
    off_vin = off_keys + (uint64_t)Q * 8;
    off_vout = off_vin + (uint64_t)Q * vs;
    off_st = off_vout + (uint64_t)Q * vs;
    off_err = (off_st + Q + 7) & ~7ull;
    bytes = off_err + 8;
    if (sealed) {
      off_tab = bytes;
      off_req = (off_tab + 4ull * (Q + 1) + 255) & ~255ull;
      off_resp = off_req + (uint64_t)Q * (32 + vs);
      bytes = off_resp + (uint64_t)Q * (24 + vs);
    }
  }
};

struct SMap {
  uint32_t id = 0;
  bolt_params p{};
  uint32_t vs = 0;
  bool sealed = false;  // BOLT_F_SEAL_CMDS: sealed requests only
  MapState state = kWaiting;
  bool closing = false;
  bool busy = false;
  bool charged = false;  // footprint counted against the budget
  int err = 0;
  uint64_t footprint = 0;
  uint64_t* h_bkeys = nullptr;  // build input in pinned host memory, until built
  uint8_t* h_bvals = nullptr;
  uint64_t n = 0;
  bolt_map* m = nullptr;
  Stage host, dev;
  uint64_t* d_bkeys = nullptr;  // build input on the device, while building
  uint8_t* d_bvals = nullptr;
  MapState retire_to = kClosed;
  std::deque<Req> queue;
};

struct Part {
  SMap* map;
  std::vector<Req> reqs;
  uint32_t q;
};

struct Group {
  uint32_t stream;
  hipEvent_t done;
  std::vector<Part> parts;
  int rc;
};

}  // namespace

struct bolt_server {
  bolt_server_params prm{};
  int device = 0;
  std::mutex mu;
  std::condition_variable cv_work;  // the loop waits here when idle
  std::condition_variable cv_done;  // clients wait here for completions
  std::thread loop;
  std::thread builder;
  std::condition_variable cv_build;  // the builder waits here for jobs
  std::vector<SMap*> build_jobs, retire_jobs;
  bool stop = false;
  std::vector<SMap*> maps;
  std::vector<hipStream_t> streams;
  std::vector<uint32_t> free_streams;
  std::vector<hipEvent_t> free_events;
  std::vector<Group*> inflight;
  std::vector<int32_t> results;  // by ticket
  uint64_t hbm_used = 0, hbm_peak = 0;
  uint64_t queued = 0;           // requests waiting (not yet launched)
  uint64_t outstanding = 0;      // requests submitted and not finished
  // statistics since the last reset
  uint64_t st_submitted = 0, st_completed = 0, st_failed = 0, st_commands = 0, st_launches = 0;
  uint64_t st_group_maps = 0, st_group_cmds = 0, st_queue_peak = 0, st_admitted = 0;
  uint64_t st_first_arr = UINT64_MAX, st_last_done = 0;
  std::vector<uint64_t> lat_ns;
};

namespace {

uint64_t map_footprint(const bolt_params* p, uint32_t Q) {
  uint64_t hbm = 0;
  if (bolt_footprint(p, &hbm, nullptr) != BOLT_OK) return 0;
  Stage s;
  s.layout(Q, p->value_bytes, (p->flags & BOLT_F_SEAL_CMDS) != 0);
  return hbm + s.bytes;
}

// Frees everything a map holds.  Builder thread (or destroy) only.
void release_map(SMap* sm) {
  if (sm->m) (void)bolt_destroy(sm->m);
  sm->m = nullptr;
  if (sm->dev.base) (void)hipFree(sm->dev.base);
  if (sm->host.base) (void)hipHostFree(sm->host.base);
  sm->dev.base = sm->host.base = nullptr;
  if (sm->d_bkeys) (void)hipFree(sm->d_bkeys);
  if (sm->d_bvals) (void)hipFree(sm->d_bvals);
  sm->d_bkeys = nullptr;
  sm->d_bvals = nullptr;
  if (sm->h_bkeys) (void)hipHostFree(sm->h_bkeys);
  if (sm->h_bvals) (void)hipHostFree(sm->h_bvals);
  sm->h_bkeys = nullptr;
  sm->h_bvals = nullptr;
}

void finish_req(bolt_server* s, const Req& r, int32_t rc, uint64_t t_done) {
  s->results[r.ticket] = rc;
  s->outstanding--;
  s->st_completed++;
  if (rc != BOLT_OK) s->st_failed++;
  s->st_commands += r.q;
  s->lat_ns.push_back(t_done > r.t_arr ? t_done - r.t_arr : 0);
  s->st_last_done = std::max(s->st_last_done, t_done);
}

// Fails every queued request of a map (it could not be admitted or broke).
void fail_queue(bolt_server* s, SMap* sm, int32_t rc) {
  const uint64_t t = now_ns();
  for (const Req& r : sm->queue) finish_req(s, r, rc, t);
  s->queued -= sm->queue.size();
  sm->queue.clear();
  s->cv_done.notify_all();
}

// Hands a map to the builder to be freed; runs under the lock.  Its share
// of the budget returns when the memory is really free.
void retire(bolt_server* s, SMap* sm, MapState to) {
  sm->state = kRetiring;
  sm->retire_to = to;
  s->retire_jobs.push_back(sm);
  s->cv_build.notify_one();
}

// Admission and retirement decisions; runs under the lock.  Returns true if
// anything changed.
bool admit(bolt_server* s) {
  bool changed = false;
  for (SMap* sm : s->maps) {
    // a closed map leaves once its last request is done
    if (sm->closing && !sm->busy && sm->queue.empty() && sm->state == kResident) {
      retire(s, sm, kClosed);
      changed = true;
    }
  }
  // admit waiting maps in the order they were opened; a map that does not
  // fit blocks the ones behind it (no overtaking, so admission is FIFO)
  for (SMap* sm : s->maps) {
    if (sm->state != kWaiting) continue;
    if (sm->closing) {  // closed before it was ever admitted
      fail_queue(s, sm, BOLT_EINVAL);
      retire(s, sm, kClosed);
      changed = true;
      continue;
    }
    if (s->prm.hbm_budget && s->hbm_used + sm->footprint > s->prm.hbm_budget) break;
    s->hbm_used += sm->footprint;
    sm->charged = true;
    s->hbm_peak = std::max(s->hbm_peak, s->hbm_used);
    s->st_admitted++;
    sm->state = kQueued;
    s->build_jobs.push_back(sm);
    s->cv_build.notify_one();
    changed = true;
  }
  return changed;
}

// Device-side set-up of one admitted map: the map, its command staging and
// its build input on the device.  Builder thread, without the lock.
int prepare(bolt_server* s, SMap* sm, hipStream_t st) {
  int rc = bolt_create(&sm->p, st, &sm->m);
  if (rc) return rc;
  const uint32_t Q = s->prm.max_batch;
  sm->host.layout(Q, sm->vs, sm->sealed);
  sm->dev.layout(Q, sm->vs, sm->sealed);
  if (hipHostMalloc((void**)&sm->host.base, sm->host.bytes, hipHostMallocDefault) != hipSuccess) return BOLT_ENOMEM;
  if (hipMalloc((void**)&sm->dev.base, sm->dev.bytes) != hipSuccess) return BOLT_ENOMEM;
  if (sm->n) {
    if (hipMalloc((void**)&sm->d_bkeys, sm->n * 8) != hipSuccess) return BOLT_ENOMEM;
    if (hipMalloc((void**)&sm->d_bvals, sm->n * sm->vs) != hipSuccess) return BOLT_ENOMEM;
    if (hipMemcpyAsync(sm->d_bkeys, sm->h_bkeys, sm->n * 8, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(sm->d_bvals, sm->h_bvals, sm->n * sm->vs, hipMemcpyHostToDevice, st) != hipSuccess)
      return BOLT_EHIP;
  }
  return BOLT_OK;
}

void run_builder(bolt_server* s) {
  (void)hipSetDevice(s->device);
  hipStream_t st = nullptr;
  (void)hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  std::unique_lock<std::mutex> lk(s->mu);
  while (!s->stop) {
    if (s->build_jobs.empty() && s->retire_jobs.empty()) {
      s->cv_build.wait(lk);
      continue;
    }
    std::vector<SMap*> builds, retires;
    builds.swap(s->build_jobs);
    retires.swap(s->retire_jobs);
    for (SMap* sm : builds) sm->state = kBuilding;
    lk.unlock();
    // frees first: they may make room for the next admissions
    for (SMap* sm : retires) release_map(sm);
    std::vector<int> rc(builds.size(), BOLT_OK);
    std::vector<bolt_map*> ms;
    std::vector<const uint64_t*> ks;
    std::vector<const void*> vs;
    std::vector<uint64_t> ns;
    std::vector<size_t> at;
    for (size_t i = 0; i < builds.size(); ++i) {
      rc[i] = prepare(s, builds[i], st);
      if (rc[i] == BOLT_OK) {
        ms.push_back(builds[i]->m);
        ks.push_back(builds[i]->d_bkeys);
        vs.push_back(builds[i]->d_bvals);
        ns.push_back(builds[i]->n);
        at.push_back(i);
      }
    }
    if (!ms.empty()) {
      int b = bolt_build_many(ms.data(), ks.data(), vs.data(), ns.data(), (uint32_t)ms.size(), st);
      if (b == BOLT_OK && hipStreamSynchronize(st) != hipSuccess) b = BOLT_EHIP;
      for (size_t j = 0; j < at.size(); ++j) {
        SMap* sm = builds[at[j]];
        rc[at[j]] = b != BOLT_OK ? b : bolt_status(sm->m);  // build errors are the map's own
        if (sm->d_bkeys) (void)hipFree(sm->d_bkeys);
        if (sm->d_bvals) (void)hipFree(sm->d_bvals);
        sm->d_bkeys = nullptr;
        sm->d_bvals = nullptr;
        if (sm->h_bkeys) (void)hipHostFree(sm->h_bkeys);
        if (sm->h_bvals) (void)hipHostFree(sm->h_bvals);
        sm->h_bkeys = nullptr;
        sm->h_bvals = nullptr;
      }
    }
    for (size_t i = 0; i < builds.size(); ++i)
      if (rc[i] != BOLT_OK) release_map(builds[i]);
    lk.lock();
    for (SMap* sm : retires) {
      if (sm->charged) s->hbm_used -= sm->footprint;
      sm->charged = false;
      sm->state = sm->retire_to;
    }
    for (size_t i = 0; i < builds.size(); ++i) {
      SMap* sm = builds[i];
      if (rc[i] == BOLT_OK) {
        sm->state = kResident;
      } else {
        sm->err = rc[i];
        fail_queue(s, sm, rc[i]);
        if (sm->charged) s->hbm_used -= sm->footprint;
        sm->charged = false;
        sm->state = kFailed;
      }
    }
    s->cv_work.notify_one();  // new residents, or room for waiting maps
    s->cv_done.notify_all();
  }
  lk.unlock();
  (void)hipStreamSynchronize(st);
  (void)hipStreamDestroy(st);
}

// Completion of launched groups; runs under the lock.
bool reap(bolt_server* s) {
  bool changed = false;
  for (size_t g = 0; g < s->inflight.size();) {
    Group* gr = s->inflight[g];
    if (hipEventQuery(gr->done) != hipSuccess) {
      ++g;
      continue;
    }
    const uint64_t t = now_ns();
    for (Part& pt : gr->parts) {
      SMap* sm = pt.map;
      int32_t rc = gr->rc;
      uint32_t dev_err = 0;
      memcpy(&dev_err, sm->host.base + sm->host.off_err, 4);
      if (rc == BOLT_OK && (dev_err & ~kErrTrace)) {
        rc = bolt_status(sm->m);  // the sticky device error of this map, as a return code
        if (rc == BOLT_OK) rc = BOLT_EHIP;
        sm->err = rc;
      }
      uint64_t at = 0;
      for (const Req& r : pt.reqs) {
        if (rc == BOLT_OK && r.rec_out) {
          memcpy(r.rec_out, sm->host.base + sm->host.off_resp + at * (24 + sm->vs), (size_t)r.q * (24 + sm->vs));
        } else if (rc == BOLT_OK) {
          memcpy(r.vout, sm->host.base + sm->host.off_vout + at * sm->vs, (size_t)r.q * sm->vs);
          memcpy(r.status, sm->host.base + sm->host.off_st + at, r.q);
        }
        at += r.q;
        finish_req(s, r, rc, t);
      }
      sm->busy = false;
      if (sm->err) {
        fail_queue(s, sm, BOLT_ESTATE);
        retire(s, sm, kFailed);
      }
    }
    s->free_streams.push_back(gr->stream);
    s->free_events.push_back(gr->done);
    delete gr;
    s->inflight[g] = s->inflight.back();
    s->inflight.pop_back();
    changed = true;
  }
  if (changed) s->cv_done.notify_all();
  return changed;
}

// One turn of continuous batching; runs under the lock.
bool launch(bolt_server* s) {
  if (s->free_streams.empty()) return false;
  std::vector<Part> parts;
  for (SMap* sm : s->maps) {
    if (sm->state != kResident || sm->busy || sm->queue.empty()) continue;
    Part pt{sm, {}, 0};
    while (!sm->queue.empty() && pt.q + sm->queue.front().q <= s->prm.max_batch) {
      pt.q += sm->queue.front().q;
      pt.reqs.push_back(sm->queue.front());
      sm->queue.pop_front();
    }
    s->queued -= pt.reqs.size();
    parts.push_back(std::move(pt));
  }
  if (parts.empty()) return false;
  const uint32_t si = s->free_streams.back();
  s->free_streams.pop_back();
  hipStream_t st = s->streams[si];
  Group* gr = new Group{si, nullptr, std::move(parts), BOLT_OK};
  if (s->free_events.empty()) {
    hipEvent_t e = nullptr;
    (void)hipEventCreateWithFlags(&e, hipEventDisableTiming);
    s->free_events.push_back(e);
  }
  gr->done = s->free_events.back();
  s->free_events.pop_back();
  std::vector<bolt_map*> ms;
  std::vector<bolt_batch> bs;
  int rc = BOLT_OK;
  for (Part& pt : gr->parts) {
    SMap* sm = pt.map;
    uint8_t* h = sm->host.base;
    memset(h + sm->host.off_err, 0, 8);
    uint8_t* d = sm->dev.base;
    uint64_t at = 0;
    if (sm->sealed) {  // command records and request starts into the staging; the device opens them
      uint32_t* tab = reinterpret_cast<uint32_t*>(h + sm->host.off_tab);
      uint32_t nreq = 0;
      for (const Req& r : pt.reqs) {
        tab[nreq++] = (uint32_t)at;
        memcpy(h + sm->host.off_req + at * (32 + sm->vs), r.rec_in, (size_t)r.q * (32 + sm->vs));
        at += r.q;
      }
      tab[nreq] = (uint32_t)at;
      if (hipMemcpyAsync(d + sm->dev.off_tab, h + sm->host.off_tab, 4ull * (nreq + 1), hipMemcpyHostToDevice, st) !=
              hipSuccess ||
          hipMemcpyAsync(d + sm->dev.off_req, h + sm->host.off_req, (size_t)pt.q * (32 + sm->vs),
                         hipMemcpyHostToDevice, st) != hipSuccess)
        rc = BOLT_EHIP;
      launch_rec_open(sm->m, d + sm->dev.off_req, pt.q, reinterpret_cast<const uint32_t*>(d + sm->dev.off_tab), nreq,
                      d, reinterpret_cast<uint64_t*>(d + sm->dev.off_keys), d + sm->dev.off_vin, st);
    } else {
      for (const Req& r : pt.reqs) {  // commands into the pinned staging, in FIFO order
        memcpy(h + at, r.ops, r.q);
        memcpy(h + sm->host.off_keys + at * 8, r.keys, (size_t)r.q * 8);
        memcpy(h + sm->host.off_vin + at * sm->vs, r.vin, (size_t)r.q * sm->vs);
        at += r.q;
      }
      // ops, keys and values in one copy each (the staging keeps them apart)
      if (hipMemcpyAsync(d, h, pt.q, hipMemcpyHostToDevice, st) != hipSuccess ||
          hipMemcpyAsync(d + sm->dev.off_keys, h + sm->host.off_keys, (size_t)pt.q * 8, hipMemcpyHostToDevice, st) !=
              hipSuccess ||
          hipMemcpyAsync(d + sm->dev.off_vin, h + sm->host.off_vin, (size_t)pt.q * sm->vs, hipMemcpyHostToDevice,
                         st) != hipSuccess)
        rc = BOLT_EHIP;
    }
    ms.push_back(sm->m);
    bs.push_back(bolt_batch{d, reinterpret_cast<const uint64_t*>(d + sm->dev.off_keys), d + sm->dev.off_vin,
                            d + sm->dev.off_vout, d + sm->dev.off_st, pt.q});
    sm->busy = true;
  }
  // a map's next group sends the pages this one rebuilds (beside its reads)
  if (rc == BOLT_OK) rc = access_many(ms.data(), bs.data(), (uint32_t)ms.size(), st, true);
  if (rc == BOLT_OK) {
    for (Part& pt : gr->parts) {
      SMap* sm = pt.map;
      uint8_t* d = sm->dev.base;
      if (sm->sealed) {  // responses sealed on the device; only their records cross to the host
        launch_rec_seal(sm->m, d + sm->dev.off_resp, pt.q, reinterpret_cast<const uint32_t*>(d + sm->dev.off_tab),
                        (uint32_t)pt.reqs.size(), d + sm->dev.off_st, d + sm->dev.off_vout, st);
        if (hipMemcpyAsync(sm->host.base + sm->host.off_resp, d + sm->dev.off_resp, (size_t)pt.q * (24 + sm->vs),
                           hipMemcpyDeviceToHost, st) != hipSuccess)
          rc = BOLT_EHIP;
      } else if (hipMemcpyAsync(sm->host.base + sm->host.off_vout, d + sm->dev.off_vout, (size_t)pt.q * sm->vs,
                                hipMemcpyDeviceToHost, st) != hipSuccess ||
                 hipMemcpyAsync(sm->host.base + sm->host.off_st, d + sm->dev.off_st, pt.q, hipMemcpyDeviceToHost,
                                st) != hipSuccess) {
        rc = BOLT_EHIP;
      }
      if (hipMemcpyAsync(sm->host.base + sm->host.off_err, &sm->m->ctl->err, 4, hipMemcpyDeviceToHost, st) !=
          hipSuccess)
        rc = BOLT_EHIP;
    }
  }
  gr->rc = rc;
  (void)hipEventRecord(gr->done, st);
  s->inflight.push_back(gr);
  s->st_launches++;
  s->st_group_maps += gr->parts.size();
  for (Part& pt : gr->parts) s->st_group_cmds += pt.q;
  return true;
}

void run_loop(bolt_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (!s->stop) {
    bool did = reap(s);
    did |= admit(s);
    did |= launch(s);
    if (did) continue;
    if (s->inflight.empty()) {
      s->cv_work.wait(lk);  // nothing in flight: sleep until a submit, open, close or build
    } else {
      // device work outstanding: poll its events, giving the lock up in between
      lk.unlock();
      std::this_thread::yield();
      lk.lock();
    }
  }
}

bool valid_ticket(bolt_server* s, uint64_t t) { return t < s->results.size(); }

}  // namespace

extern "C" {

uint64_t bolt_now_ns(void) { return now_ns(); }

int bolt_server_footprint(const bolt_params* p, uint32_t max_batch, uint64_t* bytes) {
  if (!p || !bytes) return BOLT_EINVAL;
  if (max_batch == 0) max_batch = kMaxBatch;
  if (max_batch > kMaxBatch) return BOLT_EINVAL;
  bolt_sizes z;
  int rc = bolt_sizes_of(p, &z);
  if (rc) return rc;
  *bytes = map_footprint(p, max_batch);
  return BOLT_OK;
}

int bolt_server_create(const bolt_server_params* prm, bolt_server** out) {
  if (!out) return BOLT_EINVAL;
  *out = nullptr;
  bolt_server_params p{};
  if (prm) p = *prm;
  if (p.streams == 0) p.streams = 4;
  if (p.max_batch == 0) p.max_batch = kMaxBatch;
  if (p.streams > 16 || p.max_batch > kMaxBatch || p.flags != 0) return BOLT_EINVAL;
  bolt_server* s = new (std::nothrow) bolt_server();
  if (!s) return BOLT_ENOMEM;
  s->prm = p;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return BOLT_EHIP;
  }
  for (uint32_t i = 0; i < p.streams; ++i) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
      delete s;
      return BOLT_EHIP;
    }
    s->streams.push_back(st);
    s->free_streams.push_back(p.streams - 1 - i);
  }
  std::reverse(s->free_streams.begin(), s->free_streams.end());
  s->loop = std::thread(run_loop, s);
  s->builder = std::thread(run_builder, s);
  *out = s;
  return BOLT_OK;
}

int bolt_server_open_map(bolt_server* s, const bolt_params* p, const uint64_t* host_keys, const void* host_vals,
                         uint64_t n, uint32_t* map_id) {
  if (!s || !p || !map_id) return BOLT_EINVAL;
  if (n && (!host_keys || !host_vals)) return BOLT_EINVAL;
  bolt_sizes z;
  int rc = bolt_sizes_of(p, &z);
  if (rc) return rc;
  if (n > p->capacity) return BOLT_EINVAL;
  if (p->flags & (BOLT_F_TRACE | BOLT_F_TIMING)) return BOLT_EINVAL;  // served maps keep neither
  const uint64_t fp = map_footprint(p, s->prm.max_batch);
  if (s->prm.hbm_budget && fp > s->prm.hbm_budget) return BOLT_EFULL;  // could never be admitted
  SMap* sm = new (std::nothrow) SMap();
  if (!sm) return BOLT_ENOMEM;
  sm->p = *p;
  sm->vs = p->value_bytes;
  sm->sealed = (p->flags & BOLT_F_SEAL_CMDS) != 0;
  sm->n = n;
  sm->footprint = fp;
  if (n) {  // the build input goes to pinned memory now, so its copy to the device is a plain DMA later
    if (hipHostMalloc((void**)&sm->h_bkeys, n * 8, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&sm->h_bvals, n * sm->vs, hipHostMallocDefault) != hipSuccess) {
      release_map(sm);
      delete sm;
      return BOLT_ENOMEM;
    }
    memcpy(sm->h_bkeys, host_keys, n * 8);
    memcpy(sm->h_bvals, host_vals, n * sm->vs);
  }
  {
    std::lock_guard<std::mutex> g(s->mu);
    sm->id = (uint32_t)s->maps.size();
    s->maps.push_back(sm);
  }
  s->cv_work.notify_one();
  *map_id = sm->id;
  return BOLT_OK;
}

int bolt_server_close_map(bolt_server* s, uint32_t map_id) {
  if (!s) return BOLT_EINVAL;
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (map_id >= s->maps.size() || s->maps[map_id]->closing) return BOLT_EINVAL;
    s->maps[map_id]->closing = true;
  }
  s->cv_work.notify_one();
  return BOLT_OK;
}

int bolt_server_map_state(bolt_server* s, uint32_t map_id, int* state, int* err) {
  if (!s || !state) return BOLT_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  if (map_id >= s->maps.size()) return BOLT_EINVAL;
  const SMap* sm = s->maps[map_id];
  MapState m = sm->state == kRetiring ? sm->retire_to : sm->state;
  switch (m) {
    case kWaiting: *state = BOLT_SRV_WAITING; break;
    case kQueued:
    case kBuilding: *state = BOLT_SRV_BUILDING; break;
    case kResident: *state = BOLT_SRV_RESIDENT; break;
    case kFailed: *state = BOLT_SRV_FAILED; break;
    default: *state = BOLT_SRV_CLOSED; break;
  }
  if (err) *err = sm->err;
  return BOLT_OK;
}

int bolt_server_submit(bolt_server* s, uint32_t map_id, const uint8_t* host_ops, const uint64_t* host_keys,
                       const void* host_vals_in, void* host_vals_out, uint8_t* host_status, uint32_t q,
                       uint64_t arrival_ns, uint64_t* ticket) {
  if (!s || !ticket || q == 0 || !host_ops || !host_keys || !host_vals_in || !host_vals_out || !host_status)
    return BOLT_EINVAL;
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (map_id >= s->maps.size()) return BOLT_EINVAL;
    SMap* sm = s->maps[map_id];
    if (q > s->prm.max_batch || sm->closing || sm->state == kClosed || sm->sealed) return BOLT_EINVAL;
    if (sm->err || sm->state == kFailed) return BOLT_ESTATE;
    // a bad op code would reject the whole coalesced batch: refuse it here
    for (uint32_t i = 0; i < q; ++i)
      if (host_ops[i] > BOLT_OP_DEL) return BOLT_EINVAL;
    Req r{(uint64_t)s->results.size(), host_ops, host_keys, static_cast<const uint8_t*>(host_vals_in),
          static_cast<uint8_t*>(host_vals_out), host_status, q, arrival_ns ? arrival_ns : now_ns(), nullptr,
          nullptr};
    s->results.push_back(kPending);
    sm->queue.push_back(r);
    s->queued++;
    s->outstanding++;
    s->st_submitted++;
    s->st_queue_peak = std::max(s->st_queue_peak, s->queued);
    s->st_first_arr = std::min(s->st_first_arr, r.t_arr);
    *ticket = r.ticket;
  }
  s->cv_work.notify_one();
  return BOLT_OK;
}

int bolt_server_submit_sealed(bolt_server* s, uint32_t map_id, const void* host_req_records, uint32_t q,
                              void* host_resp_records, uint64_t arrival_ns, uint64_t* ticket) {
  if (!s || !ticket || q == 0 || !host_req_records || !host_resp_records) return BOLT_EINVAL;
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (map_id >= s->maps.size()) return BOLT_EINVAL;
    SMap* sm = s->maps[map_id];
    if (q > s->prm.max_batch || sm->closing || sm->state == kClosed || !sm->sealed) return BOLT_EINVAL;
    if (sm->err || sm->state == kFailed) return BOLT_ESTATE;
    Req r{(uint64_t)s->results.size(), nullptr, nullptr, nullptr, nullptr, nullptr, q,
          arrival_ns ? arrival_ns : now_ns(), static_cast<const uint8_t*>(host_req_records),
          static_cast<uint8_t*>(host_resp_records)};
    s->results.push_back(kPending);
    sm->queue.push_back(r);
    s->queued++;
    s->outstanding++;
    s->st_submitted++;
    s->st_queue_peak = std::max(s->st_queue_peak, s->queued);
    s->st_first_arr = std::min(s->st_first_arr, r.t_arr);
    *ticket = r.ticket;
  }
  s->cv_work.notify_one();
  return BOLT_OK;
}

int bolt_server_poll(bolt_server* s, uint64_t ticket, int* result) {
  if (!s || !result) return BOLT_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  if (!valid_ticket(s, ticket)) return BOLT_EINVAL;
  *result = s->results[ticket];
  return BOLT_OK;
}

int bolt_server_wait(bolt_server* s, uint64_t ticket, uint32_t timeout_ms) {
  if (!s) return BOLT_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  if (!valid_ticket(s, ticket)) return BOLT_EINVAL;
  const bool ok = s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms),
                                      [&] { return s->results[ticket] != kPending; });
  return ok ? s->results[ticket] : BOLT_ETIMEOUT;
}

int bolt_server_drain(bolt_server* s, uint32_t timeout_ms) {
  if (!s) return BOLT_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  const bool ok =
      s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), [&] { return s->outstanding == 0; });
  return ok ? BOLT_OK : BOLT_ETIMEOUT;
}

int bolt_server_get_stats(bolt_server* s, bolt_server_stats* out) {
  if (!s || !out) return BOLT_EINVAL;
  std::vector<uint64_t> lat;
  memset(out, 0, sizeof(*out));
  {
    std::lock_guard<std::mutex> g(s->mu);
    lat = s->lat_ns;
    out->submitted = s->st_submitted;
    out->completed = s->st_completed;
    out->failed = s->st_failed;
    out->commands = s->st_commands;
    out->launches = s->st_launches;
    out->queued = s->queued;
    out->queue_peak = s->st_queue_peak;
    out->maps_admitted = s->st_admitted;
    for (SMap* sm : s->maps) {
      out->maps_resident += sm->state == kResident || sm->state == kBuilding || sm->state == kQueued;
      out->maps_waiting += sm->state == kWaiting;
    }
    out->hbm_used = s->hbm_used;
    out->hbm_peak = s->hbm_peak;
    out->mean_group_maps = s->st_launches ? (double)s->st_group_maps / s->st_launches : 0.0;
    out->mean_group_commands = s->st_launches ? (double)s->st_group_cmds / s->st_launches : 0.0;
    out->span_s = s->st_last_done > s->st_first_arr ? (s->st_last_done - s->st_first_arr) * 1e-9 : 0.0;
  }
  if (!lat.empty()) {
    std::sort(lat.begin(), lat.end());
    auto pct = [&](double f) {
      size_t i = (size_t)(f * (lat.size() - 1) + 0.5);
      return lat[std::min(i, lat.size() - 1)] * 1e-6;
    };
    out->lat_p50_ms = pct(0.50);
    out->lat_p99_ms = pct(0.99);
    out->lat_max_ms = lat.back() * 1e-6;
    double sum = 0;
    for (uint64_t v : lat) sum += (double)v;
    out->lat_mean_ms = sum / lat.size() * 1e-6;
  }
  return BOLT_OK;
}

int bolt_server_reset_stats(bolt_server* s) {
  if (!s) return BOLT_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  s->st_submitted = s->st_completed = s->st_failed = s->st_commands = s->st_launches = 0;
  s->st_group_maps = s->st_group_cmds = 0;
  s->st_queue_peak = s->queued;
  s->st_admitted = 0;
  s->st_first_arr = UINT64_MAX;
  s->st_last_done = 0;
  s->hbm_peak = s->hbm_used;
  s->lat_ns.clear();
  return BOLT_OK;
}

bolt_map* bolt_server_map(bolt_server* s, uint32_t map_id) {
  if (!s) return nullptr;
  std::lock_guard<std::mutex> g(s->mu);
  if (map_id >= s->maps.size() || s->maps[map_id]->state != kResident) return nullptr;
  return s->maps[map_id]->m;
}

int bolt_server_destroy(bolt_server* s) {
  if (!s) return BOLT_OK;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_one();
  s->cv_build.notify_one();
  if (s->loop.joinable()) s->loop.join();
  if (s->builder.joinable()) s->builder.join();
  for (hipStream_t st : s->streams) (void)hipStreamSynchronize(st);
  for (SMap* sm : s->maps) {
    release_map(sm);
    delete sm;
  }
  for (Group* g : s->inflight) {
    (void)hipEventDestroy(g->done);
    delete g;
  }
  for (hipEvent_t e : s->free_events) (void)hipEventDestroy(e);
  for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
  delete s;
  return BOLT_OK;
}

}  // extern "C"
