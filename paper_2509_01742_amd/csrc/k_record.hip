// Sealed requests: the device opens a request's command records into the
// plain command arrays the access pipeline reads, and seals the responses
// it writes (record layout and nonces in record_dev.h).  One thread per
// command.  A record that fails its tag is read as an invalid op code, so
// the whole request is rejected (nothing changes), and the map is poisoned
// with BOLT_ETAMPER, as a changed observable page poisons it.
#include "bolt_impl.h"
#include "record_dev.h"

namespace bolt {

namespace {

// Request r of the call holding command t, by binary search over the
// request starts (tab[0] = 0, tab[nreq] = q); one request when tab is null.
__device__ __forceinline__ uint32_t req_of(const uint32_t* tab, uint32_t nreq, uint32_t t) {
  if (!tab) return 0;
  uint32_t lo = 0, hi = nreq;  // tab[lo] <= t < tab[hi]
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (tab[mid] <= t) lo = mid;
    else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(64) void k_rec_open(Ctl* ctl, const uint64_t* __restrict__ recs, uint32_t q,
                                                 const uint32_t* __restrict__ tab, uint32_t nreq, uint32_t vw,
                                                 uint8_t* __restrict__ ops, uint64_t* __restrict__ keys,
                                                 uint64_t* __restrict__ vals) {
  const uint32_t t = blockIdx.x * 64 + threadIdx.x;
  if (t >= q) return;
  const uint32_t r = req_of(tab, nreq, t);
  const uint32_t i = t - (tab ? tab[r] : 0);
  const uint32_t qr = tab ? tab[r + 1] - tab[r] : q;
  const uint64_t seq = ctl->seq + 1 + r;
  uint32_t key[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) key[j] = ctl->ckey[j];
  const uint32_t words = 2 + vw;                     // plain words of a command
  const uint64_t* rec = recs + (uint64_t)t * (words + 2);  // cipher text, then the tag
  uint32_t otk[8], tag[4];
  rec_otk(key, i, seq, otk);
  rec_tag(otk, qr, words, [&](uint32_t w) { return rec[w]; }, tag);
  const uint64_t t0 = rec[words], t1 = rec[words + 1];
  const bool ok = ((uint64_t)tag[0] | ((uint64_t)tag[1] << 32)) == t0 &&
                  ((uint64_t)tag[2] | ((uint64_t)tag[3] << 32)) == t1;
  if (!ok) {
    set_err(ctl, kErrTamper);
    ops[t] = 0xFF;  // rejects the request whole
    keys[t] = 0;
    for (uint32_t w = 0; w < vw; ++w) vals[(uint64_t)t * vw + w] = 0;
    return;
  }
  RecStream ks{key, i, (uint32_t)seq, (uint32_t)(seq >> 32)};
  const uint64_t op = rec[0] ^ ks.word(0);
  ops[t] = op > 0xFF ? 0xFF : (uint8_t)op;
  keys[t] = rec[1] ^ ks.word(1);
  for (uint32_t w = 0; w < vw; ++w) vals[(uint64_t)t * vw + w] = rec[2 + w] ^ ks.word(2 + w);
}

__global__ __launch_bounds__(64) void k_rec_seal(const Ctl* ctl, uint64_t* __restrict__ out, uint32_t q,
                                                 const uint32_t* __restrict__ tab, uint32_t nreq, uint32_t vw,
                                                 const uint8_t* __restrict__ status,
                                                 const uint64_t* __restrict__ vals) {
  const uint32_t t = blockIdx.x * 64 + threadIdx.x;
  if (t >= q) return;
  const uint32_t r = req_of(tab, nreq, t);
  const uint32_t i = t - (tab ? tab[r] : 0);
  const uint32_t qr = tab ? tab[r + 1] - tab[r] : q;
  const uint64_t seq = ctl->seq + 1 + r;
  uint32_t key[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) key[j] = ctl->ckey[j];
  const uint32_t words = 1 + vw;
  uint64_t* rec = out + (uint64_t)t * (words + 2);
  RecStream ks{key, i | kRespDir, (uint32_t)seq, (uint32_t)(seq >> 32)};
  rec[0] = (uint64_t)status[t] ^ ks.word(0);
  for (uint32_t w = 0; w < vw; ++w) rec[1 + w] = vals[(uint64_t)t * vw + w] ^ ks.word(1 + w);
  uint32_t otk[8], tag[4];
  rec_otk(key, i | kRespDir, seq, otk);
  rec_tag(otk, qr, words, [&](uint32_t w) { return rec[w]; }, tag);
  rec[words] = (uint64_t)tag[0] | ((uint64_t)tag[1] << 32);
  rec[words + 1] = (uint64_t)tag[2] | ((uint64_t)tag[3] << 32);
}

// The session's request counter moves past the call's requests.
__global__ void k_rec_advance(Ctl* ctl, uint32_t nreq) { ctl->seq += nreq; }

}  // namespace

void launch_rec_open(bolt_map* m, const void* recs, uint32_t q, const uint32_t* tab, uint32_t nreq, uint8_t* ops,
                     uint64_t* keys, void* vals, hipStream_t st) {
  hipLaunchKernelGGL(k_rec_open, dim3((q + 63) / 64), dim3(64), 0, st, m->ctl, static_cast<const uint64_t*>(recs), q,
                     tab, nreq, m->s.vs / 8, ops, keys, static_cast<uint64_t*>(vals));
}

void launch_rec_seal(bolt_map* m, void* out, uint32_t q, const uint32_t* tab, uint32_t nreq, const uint8_t* status,
                     const void* vals, hipStream_t st) {
  hipLaunchKernelGGL(k_rec_seal, dim3((q + 63) / 64), dim3(64), 0, st, m->ctl, static_cast<uint64_t*>(out), q, tab,
                     nreq, m->s.vs / 8, status, static_cast<const uint64_t*>(vals));
  hipLaunchKernelGGL(k_rec_advance, dim3(1), dim3(1), 0, st, m->ctl, nreq);
}

}  // namespace bolt
