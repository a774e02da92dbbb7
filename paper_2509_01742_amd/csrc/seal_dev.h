// Device side of page sealing: ChaCha20 and Poly1305 (RFC 8439), one
// wave per page.  A sealed observable page is the ChaCha20 encryption of
// its bytes (key stream blocks 1, 2, ...) under the nonce LE32(page index)
// || LE64(write count of the page), with the Poly1305 tag of the AEAD
// construction (one-time key from block 0; tag over the cipher text, its
// padding and the two 64-bit lengths; no associated data).
#pragma once

#include "bolt_dev.h"

namespace bolt {

__host__ __device__ __forceinline__ uint32_t rotl32(uint32_t x, int n) { return __builtin_rotateleft32(x, n); }

// Orders the LDS writes of one wave's lanes before that wave's later LDS
// reads (a page staged by some lanes and read by others).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

#define BOLT_CHACHA_QR(a, b, c, d) \
  do {                             \
    a += b;                        \
    d = rotl32(d ^ a, 16);         \
    c += d;                        \
    b = rotl32(b ^ c, 12);         \
    a += b;                        \
    d = rotl32(d ^ a, 8);          \
    c += d;                        \
    b = rotl32(b ^ c, 7);          \
  } while (0)

// One ChaCha20 block (16 words): "expand 32-byte k", key, counter, nonce;
// ten double rounds; the input added back.
__host__ __device__ __forceinline__ void chacha_block(const uint32_t key[8], uint32_t counter, uint32_t n0, uint32_t n1,
                                             uint32_t n2, uint32_t out[16]) {
  const uint32_t c0 = 0x61707865u, c1 = 0x3320646eu, c2 = 0x79622d32u, c3 = 0x6b206574u;
  uint32_t x0 = c0, x1 = c1, x2 = c2, x3 = c3;
  uint32_t x4 = key[0], x5 = key[1], x6 = key[2], x7 = key[3];
  uint32_t x8 = key[4], x9 = key[5], x10 = key[6], x11 = key[7];
  uint32_t x12 = counter, x13 = n0, x14 = n1, x15 = n2;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    BOLT_CHACHA_QR(x0, x4, x8, x12);
    BOLT_CHACHA_QR(x1, x5, x9, x13);
    BOLT_CHACHA_QR(x2, x6, x10, x14);
    BOLT_CHACHA_QR(x3, x7, x11, x15);
    BOLT_CHACHA_QR(x0, x5, x10, x15);
    BOLT_CHACHA_QR(x1, x6, x11, x12);
    BOLT_CHACHA_QR(x2, x7, x8, x13);
    BOLT_CHACHA_QR(x3, x4, x9, x14);
  }
  out[0] = x0 + c0;
  out[1] = x1 + c1;
  out[2] = x2 + c2;
  out[3] = x3 + c3;
  out[4] = x4 + key[0];
  out[5] = x5 + key[1];
  out[6] = x6 + key[2];
  out[7] = x7 + key[3];
  out[8] = x8 + key[4];
  out[9] = x9 + key[5];
  out[10] = x10 + key[6];
  out[11] = x11 + key[7];
  out[12] = x12 + counter;
  out[13] = x13 + n0;
  out[14] = x14 + n1;
  out[15] = x15 + n2;
}

// ---- Poly1305 arithmetic modulo p = 2^130 - 5, five 26-bit limbs ---------

constexpr uint32_t kM26 = 0x3ffffffu;

// c = a * b mod p, partly reduced (limbs below 2^26, the second a little
// above).  Limbs of a and b below 2^28: every partial sum stays below 2^62.
__host__ __device__ __forceinline__ void fe_mul(const uint32_t a[5], const uint32_t b[5], uint32_t c[5]) {
  const uint64_t b1 = 5ull * b[1], b2 = 5ull * b[2], b3 = 5ull * b[3], b4 = 5ull * b[4];
  uint64_t d0 = (uint64_t)a[0] * b[0] + a[1] * b4 + a[2] * b3 + a[3] * b2 + a[4] * b1;
  uint64_t d1 = (uint64_t)a[0] * b[1] + (uint64_t)a[1] * b[0] + a[2] * b4 + a[3] * b3 + a[4] * b2;
  uint64_t d2 = (uint64_t)a[0] * b[2] + (uint64_t)a[1] * b[1] + (uint64_t)a[2] * b[0] + a[3] * b4 + a[4] * b3;
  uint64_t d3 = (uint64_t)a[0] * b[3] + (uint64_t)a[1] * b[2] + (uint64_t)a[2] * b[1] + (uint64_t)a[3] * b[0] +
                a[4] * b4;
  uint64_t d4 = (uint64_t)a[0] * b[4] + (uint64_t)a[1] * b[3] + (uint64_t)a[2] * b[2] + (uint64_t)a[3] * b[1] +
                (uint64_t)a[4] * b[0];
  d1 += d0 >> 26;
  d2 += d1 >> 26;
  d3 += d2 >> 26;
  d4 += d3 >> 26;
  uint64_t e0 = (d0 & kM26) + 5 * (d4 >> 26);  // 2^130 = 5 (mod p)
  c[0] = (uint32_t)(e0 & kM26);
  c[1] = (uint32_t)((d1 & kM26) + (e0 >> 26));
  c[2] = (uint32_t)(d2 & kM26);
  c[3] = (uint32_t)(d3 & kM26);
  c[4] = (uint32_t)(d4 & kM26);
}

// Four little-endian words (128 bits) as limbs, plus `top` at bit 128.
__host__ __device__ __forceinline__ void fe_from128(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3, uint32_t top,
                                           uint32_t c[5]) {
  c[0] = w0 & kM26;
  c[1] = ((w0 >> 26) | (w1 << 6)) & kM26;
  c[2] = ((w1 >> 20) | (w2 << 12)) & kM26;
  c[3] = ((w2 >> 14) | (w3 << 18)) & kM26;
  c[4] = (w3 >> 8) | (top << 24);
}

// The shuffle of a field element from another lane of the wave.
__device__ __forceinline__ void fe_shfl(const uint32_t a[5], int src, uint32_t out[5]) {
#pragma unroll
  for (int k = 0; k < 5; ++k) out[k] = (uint32_t)__shfl((int)a[k], src, 64);
}

// Poly1305 tag of `nblk` 16-byte blocks: the page's cipher text (LDS, u64
// words, `ct_words` of them) followed by the lengths block (0 || byte
// length).  One wave; every lane returns the tag.  Lane l takes the blocks
// l, l + 64, ... in Horner order with r^64, then multiplies by the power of
// r its last block still needs; r^1 .. r^64 come from a prefix product
// across the lanes; a shuffle tree sums the lanes.
__device__ __forceinline__ void poly_page_tag(const uint64_t* ct, uint32_t ct_words, const uint32_t otk[8],
                                              uint32_t tag[4]) {
  const uint32_t lane = threadIdx.x & 63;
  uint32_t r[5];
  fe_from128(otk[0] & 0x0fffffffu, otk[1] & 0x0ffffffcu, otk[2] & 0x0ffffffcu, otk[3] & 0x0ffffffcu, 0, r);
  // pw[l] = r^(l + 1) in lane l
  uint32_t pw[5] = {r[0], r[1], r[2], r[3], r[4]};
#pragma unroll
  for (int k = 1; k < 64; k <<= 1) {
    uint32_t o[5];
    fe_shfl(pw, (int)lane - k < 0 ? (int)lane : (int)lane - k, o);
    if (lane >= (uint32_t)k) {
      uint32_t t[5];
      fe_mul(pw, o, t);
#pragma unroll
      for (int j = 0; j < 5; ++j) pw[j] = t[j];
    }
  }
  uint32_t r64[5];
  fe_shfl(pw, 63, r64);
  const uint32_t nct = ct_words / 2;  // cipher-text blocks
  const uint32_t n = nct + 1;         // plus the lengths block
  uint32_t acc[5] = {0, 0, 0, 0, 0};
  int last = -1;
  for (uint32_t i = lane; i < n; i += 64) {
    uint32_t c[5];
    if (i < nct) {
      const uint64_t lo = ct[2 * i], hi = ct[2 * i + 1];
      fe_from128((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32), 1, c);
    } else {
      const uint64_t len = (uint64_t)ct_words * 8;  // aad length 0, then the cipher-text length
      fe_from128(0, 0, (uint32_t)len, (uint32_t)(len >> 32), 1, c);
    }
    if (last >= 0) {
      uint32_t t[5];
      fe_mul(acc, r64, t);
#pragma unroll
      for (int j = 0; j < 5; ++j) acc[j] = t[j];
    }
#pragma unroll
    for (int j = 0; j < 5; ++j) acc[j] += c[j];
    last = (int)i;
  }
  // weight of the lane's last block i: r^(n - i), n - i in 1..64
  const int e = last >= 0 ? (int)n - last : 1;
  uint32_t re[5];
  fe_shfl(pw, e - 1, re);
  uint64_t h[5];
  {
    uint32_t t[5];
    fe_mul(acc, re, t);
#pragma unroll
    for (int j = 0; j < 5; ++j) h[j] = last >= 0 ? t[j] : 0;
  }
#pragma unroll
  for (int k = 32; k > 0; k >>= 1) {
#pragma unroll
    for (int j = 0; j < 5; ++j) h[j] += __shfl_xor(h[j], k, 64);
  }
  // carry until every limb is below 2^26, then subtract p if h >= p
  for (int it = 0; it < 4; ++it) {
    uint64_t c = 0;
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      h[j] += c;
      c = h[j] >> 26;
      h[j] &= kM26;
    }
    h[0] += 5 * c;
  }
  uint64_t g[5], c = 5;
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    g[j] = h[j] + c;
    c = g[j] >> 26;
    g[j] &= kM26;
  }
  if (c) {
#pragma unroll
    for (int j = 0; j < 5; ++j) h[j] = g[j];
  }
  const uint64_t hlo = h[0] | (h[1] << 26) | (h[2] << 52);
  const uint64_t hhi = (h[2] >> 12) | (h[3] << 14) | (h[4] << 40);
  const uint64_t slo = (uint64_t)otk[4] | ((uint64_t)otk[5] << 32), shi = (uint64_t)otk[6] | ((uint64_t)otk[7] << 32);
  const uint64_t tlo = hlo + slo;
  const uint64_t thi = hhi + shi + (tlo < hlo ? 1 : 0);
  tag[0] = (uint32_t)tlo;
  tag[1] = (uint32_t)(tlo >> 32);
  tag[2] = (uint32_t)thi;
  tag[3] = (uint32_t)(thi >> 32);
}

// Key-stream block `lane` of a page, in one pass over the wave: lane 0's
// block 0 gives the one-time Poly1305 key (returned to every lane in otk),
// lane l >= 1 keeps block l for the page's 64-byte chunk l - 1.
__device__ __forceinline__ void chacha_first_pass(const uint32_t key[8], uint32_t n0, uint32_t n1, uint32_t n2,
                                                  uint32_t ks[16], uint32_t otk[8]) {
  const uint32_t lane = threadIdx.x & 63;
  chacha_block(key, lane, n0, n1, n2, ks);
#pragma unroll
  for (int j = 0; j < 8; ++j) otk[j] = (uint32_t)__shfl((int)ks[j], 0, 64);
}

// XOR of the page (LDS, u64 words) with its key stream, in place: chunk
// c - 1 with block c; lane l's first block (c = l) comes from the first
// pass, blocks c = l + 64, l + 128, ... of longer pages are computed here.
__device__ __forceinline__ void chacha_page_xor(uint64_t* page, uint32_t words, const uint32_t ks[16],
                                                const uint32_t key[8], uint32_t n0, uint32_t n1, uint32_t n2) {
  const uint32_t lane = threadIdx.x & 63;
  if (lane >= 1 && (lane - 1) * 8 < words) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint32_t w = (lane - 1) * 8 + j;
      if (w < words) page[w] ^= (uint64_t)ks[2 * j] | ((uint64_t)ks[2 * j + 1] << 32);
    }
  }
  for (uint32_t c = lane + 64; (c - 1) * 8 < words; c += 64) {
    uint32_t kb[16];
    chacha_block(key, c, n0, n1, n2, kb);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint32_t w = (c - 1) * 8 + j;
      if (w < words) page[w] ^= (uint64_t)kb[2 * j] | ((uint64_t)kb[2 * j + 1] << 32);
    }
  }
}

// Seals one plain page held in this wave's LDS (every lane wrote its words
// before the call): encrypts it in place under (page, write count), writes
// the cipher text to dst and returns the tag to every lane.
__device__ __forceinline__ void seal_page(uint64_t* pg, uint32_t words, const uint32_t key[8], uint32_t page,
                                          uint64_t ver, uint64_t* dst, uint32_t tag[4]) {
  const uint32_t lane = threadIdx.x & 63;
  uint32_t ks[16], otk[8];
  chacha_first_pass(key, page, (uint32_t)ver, (uint32_t)(ver >> 32), ks, otk);
  wave_sync();
  chacha_page_xor(pg, words, ks, key, page, (uint32_t)ver, (uint32_t)(ver >> 32));
  wave_sync();
  poly_page_tag(pg, words, otk, tag);
  for (uint32_t w = lane; w < words; w += 64) dst[w] = pg[w];
}

}  // namespace bolt
