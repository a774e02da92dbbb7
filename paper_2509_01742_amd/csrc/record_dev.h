// Sealed command and response records, one thread per record (the decode
// and response modules of Sec. 5.1; the user's instructions and the map's
// results cross the untrusted host only as ChaCha20-Poly1305 records,
// Sec. 3).  Record of command i of request number seq, under the session
// key:
//   plain   LE64(op) || LE64(key) || value[vs]
//   nonce   LE32(i) || LE64(seq)
//   aad     LE64(q), the request's command count
//   record  cipher text || 16-byte Poly1305 tag
// Its response: plain LE64(status) || value[vs], nonce LE32(i | 2^31) ||
// LE64(seq), the same aad.  The functions here are host-and-device: the
// device opens commands and seals responses, and the client helpers of the
// C ABI seal commands and open responses with the same code.
#pragma once

#include <stdint.h>

#include "seal_dev.h"

namespace bolt {

constexpr uint32_t kRespDir = 0x80000000u;  // nonce bit of a response record

// Poly1305 state of one thread: h accumulates in Horner order.
struct Poly1 {
  uint32_t r[5], h[5];
  __host__ __device__ void init(const uint32_t otk[8]) {
    fe_from128(otk[0] & 0x0fffffffu, otk[1] & 0x0ffffffcu, otk[2] & 0x0ffffffcu, otk[3] & 0x0ffffffcu, 0, r);
    for (int j = 0; j < 5; ++j) h[j] = 0;
  }
  // one full 16-byte block (the 2^128 bit set)
  __host__ __device__ void block(uint64_t lo, uint64_t hi) {
    uint32_t c[5], t[5];
    fe_from128((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32), 1, c);
    for (int j = 0; j < 5; ++j) h[j] += c[j];
    fe_mul(h, r, t);
    for (int j = 0; j < 5; ++j) h[j] = t[j];
  }
  // h reduced modulo 2^130 - 5, plus s, as four LE words
  __host__ __device__ void finish(const uint32_t otk[8], uint32_t tag[4]) const {
    uint64_t x[5];
    for (int j = 0; j < 5; ++j) x[j] = h[j];
    for (int it = 0; it < 2; ++it) {
      uint64_t c = 0;
      for (int j = 0; j < 5; ++j) {
        x[j] += c;
        c = x[j] >> 26;
        x[j] &= kM26;
      }
      x[0] += 5 * c;
    }
    uint64_t g[5], c = 5;
    for (int j = 0; j < 5; ++j) {
      g[j] = x[j] + c;
      c = g[j] >> 26;
      g[j] &= kM26;
    }
    if (c)
      for (int j = 0; j < 5; ++j) x[j] = g[j];
    const uint64_t hlo = x[0] | (x[1] << 26) | (x[2] << 52);
    const uint64_t hhi = (x[2] >> 12) | (x[3] << 14) | (x[4] << 40);
    const uint64_t slo = (uint64_t)otk[4] | ((uint64_t)otk[5] << 32);
    const uint64_t shi = (uint64_t)otk[6] | ((uint64_t)otk[7] << 32);
    const uint64_t tlo = hlo + slo;
    const uint64_t thi = hhi + shi + (tlo < hlo ? 1 : 0);
    tag[0] = (uint32_t)tlo;
    tag[1] = (uint32_t)(tlo >> 32);
    tag[2] = (uint32_t)thi;
    tag[3] = (uint32_t)(thi >> 32);
  }
};

// Key-stream word w (64 bits) of a record: block 1 + w / 8.
struct RecStream {
  const uint32_t* key;
  uint32_t n0, n1, n2;
  uint32_t blk = 0xffffffffu;
  uint32_t ks[16];
  __host__ __device__ uint64_t word(uint32_t w) {
    const uint32_t b = 1 + w / 8;
    if (b != blk) {
      chacha_block(key, b, n0, n1, n2, ks);
      blk = b;
    }
    const uint32_t j = w % 8;
    return (uint64_t)ks[2 * j] | ((uint64_t)ks[2 * j + 1] << 32);
  }
};

// Tag of a record's cipher text (words ct(0..words-1), read through `ct`)
// with aad LE64(q).
template <class CT>
__host__ __device__ void rec_tag(const uint32_t otk[8], uint64_t q, uint32_t words, CT ct, uint32_t tag[4]) {
  Poly1 p;
  p.init(otk);
  p.block(q, 0);  // the 8-byte aad, zero-padded to 16
  for (uint32_t w = 0; w < words; w += 2) p.block(ct(w), w + 1 < words ? ct(w + 1) : 0);
  p.block(8, (uint64_t)words * 8);  // LE64(aad length) || LE64(cipher-text length)
  p.finish(otk, tag);
}

// The one-time Poly1305 key of a record: ChaCha20 block 0.
__host__ __device__ inline void rec_otk(const uint32_t key[8], uint32_t n0, uint64_t seq, uint32_t otk[8]) {
  uint32_t b0[16];
  chacha_block(key, 0, n0, (uint32_t)seq, (uint32_t)(seq >> 32), b0);
  for (int j = 0; j < 8; ++j) otk[j] = b0[j];
}

}  // namespace bolt
