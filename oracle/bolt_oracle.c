/*
 * Reference oracle for the BOLT oblivious map (arxiv 2509.01742).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this file.  The product library
 * never links, loads or calls it.  It shares no code with the HIP library:
 * the PRF, the two networks and the map procedure are written separately
 * here, plainly and single-threaded, so that the two can be compared
 * element by element.
 *
 * Contents
 *   1. BLAKE2s-256 with a key (RFC 7693).  It is the keyed PRF that stands in
 *      for the unnamed hash of Sec. 5.1 step 3 and for random_remap() of
 *      Alg. 1.
 *   1b, 1c. ChaCha20-Poly1305 (RFC 8439), which seals observable pages
 *      and the command and response records of sealed requests.
 *   2. Parameter derivation: bins (Sec. 4.1), bin capacity (Claim 4.2), stash
 *      bound (Claim 4.4), position-map rows (Sec. 5.2, "decomposed HBM
 *      storage").
 *   3. A scalar bitonic sorting network and a scalar shift network
 *      (order-preserving compaction and its inverse, expansion).
 *   4. The map: the build (the "fast data initialization" of Sec. 5.2, done
 *      as an oblivious procedure) and batched access (Alg. 1 with the module
 *      order of Sec. 5.1).  Every access to the observable store goes
 *      through one pair of functions that also records it.
 *   5. The plain definition of the answers (O1) as a C hash table, the
 *      timed plain baseline.
 *
 * Built with -fopenmp, the same source is the parallel CPU baseline of the
 * same procedure: the loops whose iterations are independent (the network
 * stages, the PRFs of a build or a batch, the placement choices of a round,
 * the page write-out when no trace is kept) carry OpenMP pragmas, which the
 * plain single-thread build ignores.  The results do not depend on it (the
 * tests compare the two builds).
 *
 * Readings of points where the paper is silent (all listed in the design
 * notes of the repository):
 *   - PRF = keyed BLAKE2s; input = domain byte || LE64(x); output = four
 *     little-endian 64-bit words w0..w3.  Domain 1 = a key's two bins,
 *     domain 2 = a key's position-map rows, domain 3 = the per-step tape.
 *   - A pair of distinct bins from (w0, w1): p1 = hi64(w0 * B),
 *     p2 = (p1 + 1 + hi64(w1 * (B - 1))) mod B.  This is uniform over the
 *     B(B-1) ordered pairs up to a bias below B / 2^64 (Claim 4.1 proof).
 *   - Bins [0, K) live in HBM, bins [K, B) are observable pages 0..M-1.
 *   - Page = u64 valid mask || keys[Z] || values[Z][vs] || zero pad to a
 *     multiple of 128 bytes.  Real items come first, sorted by key; dummy
 *     slots are zero.  HBM bins use the same format.
 *   - P2C: the second bin wins only when strictly less loaded.  The load of a
 *     bin counts its stash items too.
 *   - Build placement runs in rounds of ceil(B/16) keys in input order, each
 *     round seeing the loads at its start.  Position-map inserts run in
 *     rounds of ceil(R_pm/16) with the same rule over d = 4 rows, ties to
 *     the lowest choice.
 *   - Batch semantics: answers equal the sequential semantics.  The first
 *     occurrence of a key in a batch (its leader) reads its mapped pair;
 *     every other occurrence, and every miss, reads the fresh pair F(s) of
 *     its step s.  Every key present at the end of the batch is remapped
 *     once, with the pair R(s) of its leader's step, by P2C over the loads
 *     left after all removals, in rounds of ceil(B/16) leaders in op order.
 *     Remapping comes before write-back (Sec. 5.1 step 5), and each distinct
 *     page read in the batch is written back once, in ascending order,
 *     holding its survivors plus every stash item destined for it.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* 1. BLAKE2s-256 (RFC 7693, Sec. 2 and 3)                              */
/* ------------------------------------------------------------------ */

static const uint32_t OR_B2S_IV[8] = {
    0x6A09E667u, 0xBB67AE85u, 0x3C6EF372u, 0xA54FF53Au,
    0x510E527Fu, 0x9B05688Cu, 0x1F83D9ABu, 0x5BE0CD19u};

static const uint8_t OR_B2S_SIGMA[10][16] = {
    {0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15},
    {14, 10, 4, 8, 9, 15, 13, 6, 1, 12, 0, 2, 11, 7, 5, 3},
    {11, 8, 12, 0, 5, 2, 15, 13, 10, 14, 3, 6, 7, 1, 9, 4},
    {7, 9, 3, 1, 13, 12, 11, 14, 2, 6, 5, 10, 4, 0, 15, 8},
    {9, 0, 5, 7, 2, 4, 10, 15, 14, 1, 11, 12, 6, 8, 3, 13},
    {2, 12, 6, 10, 0, 11, 8, 3, 4, 13, 7, 5, 15, 14, 1, 9},
    {12, 5, 1, 15, 14, 13, 4, 10, 0, 7, 6, 3, 9, 2, 8, 11},
    {13, 11, 7, 14, 12, 1, 3, 9, 5, 0, 15, 4, 8, 6, 2, 10},
    {6, 15, 14, 9, 11, 3, 0, 8, 12, 2, 13, 7, 1, 4, 10, 5},
    {10, 2, 8, 4, 7, 6, 1, 5, 15, 11, 9, 14, 3, 12, 13, 0}};

static uint32_t or_rotr32(uint32_t x, int n) { return (x >> n) | (x << (32 - n)); }

static uint32_t or_le32(const uint8_t* p) {
  return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}

static uint64_t or_le64(const uint8_t* p) {
  uint64_t v = 0;
  for (int i = 7; i >= 0; --i) v = (v << 8) | p[i];
  return v;
}

static void or_put_le64(uint8_t* p, uint64_t v) {
  for (int i = 0; i < 8; ++i) p[i] = (uint8_t)(v >> (8 * i));
}

/* The mixing function G (RFC 7693 Sec. 3.1) with BLAKE2s rotations. */
static void or_b2s_g(uint32_t v[16], int a, int b, int c, int d, uint32_t x, uint32_t y) {
  v[a] = v[a] + v[b] + x;
  v[d] = or_rotr32(v[d] ^ v[a], 16);
  v[c] = v[c] + v[d];
  v[b] = or_rotr32(v[b] ^ v[c], 12);
  v[a] = v[a] + v[b] + y;
  v[d] = or_rotr32(v[d] ^ v[a], 8);
  v[c] = v[c] + v[d];
  v[b] = or_rotr32(v[b] ^ v[c], 7);
}

/* The compression function F (RFC 7693 Sec. 3.2). */
static void or_b2s_compress(uint32_t h[8], const uint8_t block[64], uint64_t t, int last) {
  uint32_t v[16], m[16];
  for (int i = 0; i < 16; ++i) m[i] = or_le32(block + 4 * i);
  for (int i = 0; i < 8; ++i) {
    v[i] = h[i];
    v[i + 8] = OR_B2S_IV[i];
  }
  v[12] ^= (uint32_t)t;
  v[13] ^= (uint32_t)(t >> 32);
  if (last) v[14] = ~v[14];
  for (int r = 0; r < 10; ++r) {
    const uint8_t* s = OR_B2S_SIGMA[r];
    or_b2s_g(v, 0, 4, 8, 12, m[s[0]], m[s[1]]);
    or_b2s_g(v, 1, 5, 9, 13, m[s[2]], m[s[3]]);
    or_b2s_g(v, 2, 6, 10, 14, m[s[4]], m[s[5]]);
    or_b2s_g(v, 3, 7, 11, 15, m[s[6]], m[s[7]]);
    or_b2s_g(v, 0, 5, 10, 15, m[s[8]], m[s[9]]);
    or_b2s_g(v, 1, 6, 11, 12, m[s[10]], m[s[11]]);
    or_b2s_g(v, 2, 7, 8, 13, m[s[12]], m[s[13]]);
    or_b2s_g(v, 3, 4, 9, 14, m[s[14]], m[s[15]]);
  }
  for (int i = 0; i < 8; ++i) h[i] ^= v[i] ^ v[i + 8];
}

/* BLAKE2s with digest length nn (1..32) and key length kk (0..32): the
 * key, padded to one block, is processed first (RFC 7693 Sec. 3.3). */
int or_blake2s(uint8_t* out, uint32_t nn, const uint8_t* key, uint32_t kk, const uint8_t* msg, uint64_t ll) {
  if (nn < 1 || nn > 32 || kk > 32) return -1;
  uint32_t h[8];
  for (int i = 0; i < 8; ++i) h[i] = OR_B2S_IV[i];
  h[0] ^= 0x01010000u ^ (kk << 8) ^ nn;
  uint64_t total = (kk ? 64u : 0u) + ll;
  uint64_t nblocks = total == 0 ? 1 : (total + 63) / 64;
  for (uint64_t b = 0; b < nblocks; ++b) {
    uint8_t block[64];
    memset(block, 0, 64);
    for (uint64_t i = 0; i < 64; ++i) {
      uint64_t pos = 64 * b + i; /* position in key block || message */
      if (pos >= total) break;
      if (kk && pos < 64)
        block[i] = pos < kk ? key[pos] : 0;
      else
        block[i] = msg[pos - (kk ? 64 : 0)];
    }
    uint64_t t = 64 * (b + 1) < total ? 64 * (b + 1) : total;
    or_b2s_compress(h, block, t, b + 1 == nblocks);
  }
  uint8_t full[32];
  for (int i = 0; i < 8; ++i) {
    full[4 * i + 0] = (uint8_t)h[i];
    full[4 * i + 1] = (uint8_t)(h[i] >> 8);
    full[4 * i + 2] = (uint8_t)(h[i] >> 16);
    full[4 * i + 3] = (uint8_t)(h[i] >> 24);
  }
  memcpy(out, full, nn);
  return 0;
}

/* PRF_K(domain, x) -> four 64-bit words. */
void or_prf(const uint8_t key[32], uint8_t domain, uint64_t x, uint64_t w[4]) {
  uint8_t msg[9], out[32];
  msg[0] = domain;
  or_put_le64(msg + 1, x);
  or_blake2s(out, 32, key, 32, msg, 9);
  for (int j = 0; j < 4; ++j) w[j] = or_le64(out + 8 * j);
}

static uint64_t or_mulhi(uint64_t a, uint64_t b) {
  return (uint64_t)(((unsigned __int128)a * (unsigned __int128)b) >> 64);
}

/* An ordered pair of distinct bins in [0, B) from two PRF words. */
void or_pair(uint64_t w0, uint64_t w1, uint64_t B, uint32_t* p1, uint32_t* p2) {
  uint64_t a = or_mulhi(w0, B);
  uint64_t b = (a + 1 + or_mulhi(w1, B - 1)) % B;
  *p1 = (uint32_t)a;
  *p2 = (uint32_t)b;
}

/* ------------------------------------------------------------------ */
/* 1b. ChaCha20 and Poly1305 (RFC 8439): the authenticated encryption   */
/*     that seals observable pages (the paper assumes pages encrypted   */
/*     with authentication, Sec. 3 and Sec. 5.1 step 4).                */
/* ------------------------------------------------------------------ */

static uint32_t or_rotl32(uint32_t x, int n) { return (x << n) | (x >> (32 - n)); }

/* The ChaCha quarter round on four words of the state (RFC 8439, 2.1). */
static void or_quarter(uint32_t* s, int a, int b, int c, int d) {
  s[a] += s[b]; s[d] ^= s[a]; s[d] = or_rotl32(s[d], 16);
  s[c] += s[d]; s[b] ^= s[c]; s[b] = or_rotl32(s[b], 12);
  s[a] += s[b]; s[d] ^= s[a]; s[d] = or_rotl32(s[d], 8);
  s[c] += s[d]; s[b] ^= s[c]; s[b] = or_rotl32(s[b], 7);
}

/* One 64-byte ChaCha20 block: constants, key, block counter, nonce; ten
 * double rounds (columns, then diagonals); the input added back (2.3). */
void or_chacha20_block(const uint8_t key[32], uint32_t counter, const uint8_t nonce[12], uint8_t out[64]) {
  uint32_t in[16], x[16];
  in[0] = 0x61707865u; in[1] = 0x3320646eu; in[2] = 0x79622d32u; in[3] = 0x6b206574u; /* "expand 32-byte k" */
  for (int i = 0; i < 8; ++i) in[4 + i] = or_le32(key + 4 * i);
  in[12] = counter;
  for (int i = 0; i < 3; ++i) in[13 + i] = or_le32(nonce + 4 * i);
  memcpy(x, in, sizeof(x));
  for (int r = 0; r < 10; ++r) {
    or_quarter(x, 0, 4, 8, 12); or_quarter(x, 1, 5, 9, 13); or_quarter(x, 2, 6, 10, 14); or_quarter(x, 3, 7, 11, 15);
    or_quarter(x, 0, 5, 10, 15); or_quarter(x, 1, 6, 11, 12); or_quarter(x, 2, 7, 8, 13); or_quarter(x, 3, 4, 9, 14);
  }
  for (int i = 0; i < 16; ++i) {
    const uint32_t v = x[i] + in[i];
    out[4 * i] = (uint8_t)v; out[4 * i + 1] = (uint8_t)(v >> 8);
    out[4 * i + 2] = (uint8_t)(v >> 16); out[4 * i + 3] = (uint8_t)(v >> 24);
  }
}

/* data XOR the key stream of blocks counter, counter + 1, ... (2.4). */
static void or_chacha20_xor(const uint8_t key[32], uint32_t counter, const uint8_t nonce[12], const uint8_t* in,
                            uint8_t* out, uint64_t len) {
  uint8_t ks[64];
  for (uint64_t off = 0; off < len; off += 64, ++counter) {
    or_chacha20_block(key, counter, nonce, ks);
    for (uint64_t j = 0; j < 64 && off + j < len; ++j) out[off + j] = in[off + j] ^ ks[j];
  }
}

/* Poly1305 (2.5): h = (h + block + 2^(8 len)) * r mod 2^130 - 5 over the
 * 16-byte blocks, then tag = (h + s) mod 2^128.  Numbers in five 26-bit
 * limbs; products folded with 2^130 = 5 (mod p). */
void or_poly1305(const uint8_t key[32], const uint8_t* msg, uint64_t len, uint8_t tag[16]) {
  const uint32_t M26 = 0x3ffffff;
  uint8_t rb[16];
  memcpy(rb, key, 16);
  rb[3] &= 15; rb[7] &= 15; rb[11] &= 15; rb[15] &= 15; /* clamp */
  rb[4] &= 252; rb[8] &= 252; rb[12] &= 252;
  uint64_t rlo = or_le64(rb), rhi = or_le64(rb + 8);
  uint64_t r[5] = {rlo & M26, (rlo >> 26) & M26, ((rlo >> 52) | (rhi << 12)) & M26, (rhi >> 14) & M26, rhi >> 40};
  uint64_t h[5] = {0, 0, 0, 0, 0};
  for (uint64_t off = 0; off < len; off += 16) {
    uint8_t blk[17] = {0};
    const uint64_t n = len - off < 16 ? len - off : 16;
    memcpy(blk, msg + off, n);
    blk[n] = 1; /* the bit just above the block's bytes */
    const uint64_t lo = or_le64(blk), mi = or_le64(blk + 8), top = blk[16];
    h[0] += lo & M26;
    h[1] += (lo >> 26) & M26;
    h[2] += ((lo >> 52) | (mi << 12)) & M26;
    h[3] += (mi >> 14) & M26;
    h[4] += (mi >> 40) | (top << 24);
    uint64_t d[9] = {0};
    for (int i = 0; i < 5; ++i)
      for (int j = 0; j < 5; ++j) d[i + j] += h[i] * r[j];
    for (int k = 8; k >= 5; --k) d[k - 5] += 5 * d[k]; /* 2^130 = 5 mod p */
    uint64_t c = 0;
    for (int k = 0; k < 5; ++k) {
      d[k] += c;
      c = d[k] >> 26;
      h[k] = d[k] & M26;
    }
    h[0] += 5 * c;
    h[1] += h[0] >> 26;
    h[0] &= M26;
  }
  /* carry until every limb is below 2^26 (h < 2^130), then h mod p:
   * subtract p when h >= p, that is when h + 5 reaches 2^130 */
  uint64_t c = 0;
  for (int it = 0; it < 4; ++it) {
    c = 0;
    for (int k = 0; k < 5; ++k) {
      h[k] += c;
      c = h[k] >> 26;
      h[k] &= M26;
    }
    h[0] += 5 * c;
  }
  uint64_t g[5];
  c = 5;
  for (int k = 0; k < 5; ++k) {
    g[k] = h[k] + c;
    c = g[k] >> 26;
    g[k] &= M26;
  }
  if (c) memcpy(h, g, sizeof(h)); /* h + 5 reached 2^130: h >= p */
  const uint64_t hlo = h[0] | (h[1] << 26) | (h[2] << 52);
  const uint64_t hhi = (h[2] >> 12) | (h[3] << 14) | (h[4] << 40);
  const uint64_t slo = or_le64(key + 16), shi = or_le64(key + 24);
  const uint64_t tlo = hlo + slo;
  const uint64_t thi = hhi + shi + (tlo < hlo);
  or_put_le64(tag, tlo);
  or_put_le64(tag + 8, thi);
}

/* AEAD_CHACHA20_POLY1305 (2.8): one-time Poly1305 key from block 0, text
 * encrypted from block 1, tag over aad || pad || ct || pad || LE64 lengths. */
static void or_aead_mac(const uint8_t key[32], const uint8_t nonce[12], const uint8_t* aad, uint64_t aad_len,
                        const uint8_t* ct, uint64_t len, uint8_t tag[16]) {
  uint8_t blk0[64];
  or_chacha20_block(key, 0, nonce, blk0);
  const uint64_t pa = (aad_len + 15) / 16 * 16, pc = (len + 15) / 16 * 16;
  uint8_t* mac = calloc(pa + pc + 16, 1);
  if (aad_len) memcpy(mac, aad, aad_len);
  if (len) memcpy(mac + pa, ct, len);
  or_put_le64(mac + pa + pc, aad_len);
  or_put_le64(mac + pa + pc + 8, len);
  or_poly1305(blk0, mac, pa + pc + 16, tag);
  free(mac);
}

void or_aead_seal(const uint8_t key[32], const uint8_t nonce[12], const uint8_t* aad, uint64_t aad_len,
                  const uint8_t* pt, uint64_t len, uint8_t* ct, uint8_t tag[16]) {
  or_chacha20_xor(key, 1, nonce, pt, ct, len);
  or_aead_mac(key, nonce, aad, aad_len, ct, len, tag);
}

/* 0 and the plain text when the tag checks, -1 (and nothing written) when not. */
int or_aead_open(const uint8_t key[32], const uint8_t nonce[12], const uint8_t* aad, uint64_t aad_len,
                 const uint8_t* ct, uint64_t len, const uint8_t tag[16], uint8_t* pt) {
  uint8_t want[16];
  or_aead_mac(key, nonce, aad, aad_len, ct, len, want);
  uint8_t diff = 0;
  for (int i = 0; i < 16; ++i) diff |= (uint8_t)(want[i] ^ tag[i]);
  if (diff) return -1;
  or_chacha20_xor(key, 1, nonce, ct, pt, len);
  return 0;
}

/* ------------------------------------------------------------------ */
/* 1c. Sealed command and response records                              */
/* ------------------------------------------------------------------ */

/* The user's instructions reach the map encrypted, and its results leave
 * encrypted (Sec. 3, threat model: the host only relays them; Sec. 5.1,
 * the decode module opens instructions, the response module seals
 * results).  Every command and every response is its own fixed-length
 * ChaCha20-Poly1305 record under the session key:
 *   command i of request seq:  plain  LE64(op) || LE64(key) || value[vs]
 *                              nonce  LE32(i) || LE64(seq)
 *   its response:              plain  LE64(status) || value[vs]
 *                              nonce  LE32(i | 2^31) || LE64(seq)
 *   associated data of both:   LE64(q), the request's command count
 *   record                     cipher text || 16-byte tag
 * Requests of a session are numbered 1, 2, ... in the order the map runs
 * them, so a replayed, reordered, truncated or changed request fails its
 * tags. */

static void or_rec_nonce(uint32_t dir, uint32_t i, uint64_t seq, uint8_t nonce[12]) {
  uint32_t w = i | (dir << 31);
  nonce[0] = (uint8_t)w; nonce[1] = (uint8_t)(w >> 8); nonce[2] = (uint8_t)(w >> 16); nonce[3] = (uint8_t)(w >> 24);
  or_put_le64(nonce + 4, seq);
}

/* Seals q commands into q records of 32 + vs bytes (the client's side). */
void or_cmd_seal(const uint8_t key[32], uint64_t seq, uint32_t q, uint32_t vs, const uint8_t* ops,
                 const uint64_t* keys, const uint8_t* vals, uint8_t* out) {
  uint8_t aad[8], nonce[12];
  or_put_le64(aad, q);
  uint8_t* plain = malloc(16 + vs);
  for (uint32_t i = 0; i < q; ++i) {
    or_put_le64(plain, ops[i]);
    or_put_le64(plain + 8, keys[i]);
    memcpy(plain + 16, vals + (size_t)i * vs, vs);
    or_rec_nonce(0, i, seq, nonce);
    uint8_t* rec = out + (size_t)i * (32 + vs);
    or_aead_seal(key, nonce, aad, 8, plain, 16 + vs, rec, rec + 16 + vs);
  }
  free(plain);
}

/* Opens q command records; returns how many failed their tag (their
 * fields are then zero, with op 0xFF). */
uint32_t or_cmd_open(const uint8_t key[32], uint64_t seq, uint32_t q, uint32_t vs, const uint8_t* recs,
                     uint8_t* ops, uint64_t* keys, uint8_t* vals) {
  uint8_t aad[8], nonce[12];
  or_put_le64(aad, q);
  uint8_t* plain = malloc(16 + vs);
  uint32_t bad = 0;
  for (uint32_t i = 0; i < q; ++i) {
    const uint8_t* rec = recs + (size_t)i * (32 + vs);
    or_rec_nonce(0, i, seq, nonce);
    if (or_aead_open(key, nonce, aad, 8, rec, 16 + vs, rec + 16 + vs, plain)) {
      bad++;
      ops[i] = 0xFF;
      keys[i] = 0;
      memset(vals + (size_t)i * vs, 0, vs);
      continue;
    }
    uint64_t op = or_le64(plain);
    ops[i] = op > 0xFF ? 0xFF : (uint8_t)op;
    keys[i] = or_le64(plain + 8);
    memcpy(vals + (size_t)i * vs, plain + 16, vs);
  }
  free(plain);
  return bad;
}

/* Seals q responses into q records of 24 + vs bytes (the map's side). */
void or_resp_seal(const uint8_t key[32], uint64_t seq, uint32_t q, uint32_t vs, const uint8_t* status,
                  const uint8_t* vals, uint8_t* out) {
  uint8_t aad[8], nonce[12];
  or_put_le64(aad, q);
  uint8_t* plain = malloc(8 + vs);
  for (uint32_t i = 0; i < q; ++i) {
    or_put_le64(plain, status[i]);
    memcpy(plain + 8, vals + (size_t)i * vs, vs);
    or_rec_nonce(1, i, seq, nonce);
    uint8_t* rec = out + (size_t)i * (24 + vs);
    or_aead_seal(key, nonce, aad, 8, plain, 8 + vs, rec, rec + 8 + vs);
  }
  free(plain);
}

/* Opens q response records (the client's side); returns the failures. */
uint32_t or_resp_open(const uint8_t key[32], uint64_t seq, uint32_t q, uint32_t vs, const uint8_t* recs,
                      uint8_t* status, uint8_t* vals) {
  uint8_t aad[8], nonce[12];
  or_put_le64(aad, q);
  uint8_t* plain = malloc(8 + vs);
  uint32_t bad = 0;
  for (uint32_t i = 0; i < q; ++i) {
    const uint8_t* rec = recs + (size_t)i * (24 + vs);
    or_rec_nonce(1, i, seq, nonce);
    if (or_aead_open(key, nonce, aad, 8, rec, 8 + vs, rec + 8 + vs, plain)) {
      bad++;
      status[i] = 0;
      memset(vals + (size_t)i * vs, 0, vs);
      continue;
    }
    status[i] = (uint8_t)or_le64(plain);
    memcpy(vals + (size_t)i * vs, plain + 8, vs);
  }
  free(plain);
  return bad;
}

/* ------------------------------------------------------------------ */
/* 2. Parameters                                                        */
/* ------------------------------------------------------------------ */

typedef struct {
  uint64_t cap;        /* N_max, the most live keys */
  uint32_t vs;         /* value bytes */
  uint32_t c;          /* mean bin load N/(K+M) (Claim 4.2) */
  uint32_t alpha_pm;   /* alpha = K/(K+M) in per-mille (Claim 4.4) */
  uint32_t Z;          /* bin capacity = l_max (Claim 4.2) */
  uint32_t d;          /* position-map choices (Sec. 5.2) */
  uint32_t kpr;        /* keys per position-map row, N/R_pm (Sec. 5.2) */
  uint32_t W;          /* slots per position-map row */
  uint64_t B, K, M;    /* bins, HBM bins, host pages */
  uint64_t R_pm;       /* position-map rows */
  uint64_t page_bytes; /* bytes per page and per HBM bin */
  uint64_t stash_bound;/* Claim 4.4 with the O() constant set to 1 */
  uint32_t lmax;       /* l_max of Claim 4.2 with the O() constant set to 1 */
  uint64_t hbm_bound;  /* Claim 4.3 with the O() constant set to 1: items the K HBM bins may hold */
} or_sizes;

static uint32_t or_ceil_log2(uint64_t x) {
  uint32_t l = 0;
  while ((1ull << l) < x) ++l;
  return l;
}

/* Claim 4.4: (1+alpha) M / 2 + l_max * sqrt(M ln N), rounded up. */
uint64_t or_stash_bound(uint64_t M, uint32_t alpha_pm, uint32_t Z, uint64_t cap) {
  double a = (double)alpha_pm / 1000.0;
  double x = (1.0 + a) * (double)M / 2.0 + (double)Z * sqrt((double)M * log((double)cap));
  return (uint64_t)ceil(x);
}

/* Claim 4.3: sum of HBM bin loads <= K c + l_max sqrt(K ln N). */
double or_claim43_bound(double K, double c, double lmax, double N) { return K * c + lmax * sqrt(K * log(N)); }

/* Claim 4.4 with real-valued M and alpha. */
double or_claim44_bound(double M, double alpha, double lmax, double N) {
  return (1.0 + alpha) * M / 2.0 + lmax * sqrt(M * log(N));
}

/* Claim 5.2: HBM bits = (beta1 + beta2) vs + (2 log2 N + ks)(N + R log2 log2 N / log2 d),
 * with R the position-map rows; ks and vs in bits. */
double or_claim52_bits(double N, double ks, double vs, double beta1, double beta2, double R, double d) {
  return (beta1 + beta2) * vs + (2.0 * log2(N) + ks) * (N + R * log2(log2(N)) / log2(d));
}

int or_sizing(uint64_t cap, uint32_t vs, uint32_t c, uint32_t alpha_pm, uint32_t bin_slots,
              uint32_t d, uint32_t kpr, uint32_t W, or_sizes* s) {
  if (cap < 2 || vs == 0 || vs % 8 || vs > 4096 || c == 0 || alpha_pm >= 1000) return -1;
  if (d == 0 || d > 4 || kpr == 0 || W == 0 || W > 32) return -1;
  memset(s, 0, sizeof(*s));
  s->cap = cap;
  s->vs = vs;
  s->c = c;
  s->alpha_pm = alpha_pm;
  s->d = d;
  s->kpr = kpr;
  s->W = W;
  s->B = (cap + c - 1) / c; /* N = c (K + M), Claim 4.2 */
  if (s->B < 2) return -1;
  s->K = (uint64_t)alpha_pm * s->B / 1000;
  s->M = s->B - s->K;
  /* l_max = c + O(log2 log2 N) with the constant 1 (Claim 4.2). */
  s->lmax = c + or_ceil_log2(or_ceil_log2(cap)) + 1;
  /* The default capacity is l_max, plus one slot when a batch can fill a
   * sizeable part of a placement round: batches place their keys in rounds
   * that all see the loads at the round's start, and a round of B/64 keys
   * or more (B <= 64 * 8192, the largest batch) lifts the tail of the bin
   * loads by one over one-at-a-time placement. */
  s->Z = bin_slots ? bin_slots : s->lmax + (s->B <= 64ull * 8192 ? 1 : 0);
  if (s->Z == 0 || s->Z > 64) return -1;
  s->R_pm = (cap + kpr - 1) / kpr;
  uint64_t raw = 8 + 8ull * s->Z + (uint64_t)vs * s->Z;
  s->page_bytes = (raw + 127) / 128 * 128;
  s->stash_bound = or_stash_bound(s->M, alpha_pm, s->lmax, cap);
  s->hbm_bound = (uint64_t)ceil(or_claim43_bound((double)s->K, (double)c, (double)s->lmax, (double)cap));
  return 0;
}

/* ------------------------------------------------------------------ */
/* 3. Networks                                                          */
/* ------------------------------------------------------------------ */

/* Bitonic sorting network, ascending, n a power of two.  Stage (k, j)
 * compares element i with element i ^ j; the block of size k that holds i
 * sorts ascending when bit k of i is clear.  Every stage touches every
 * element whatever the data. */
int or_bitonic_sort_u64(uint64_t* a, uint64_t n) {
  if (n & (n - 1)) return -1;
  for (uint64_t k = 2; k <= n; k <<= 1)
    for (uint64_t j = k >> 1; j > 0; j >>= 1)
#pragma omp parallel for if (n >= 4096)
      for (uint64_t i = 0; i < n; ++i) {
        uint64_t l = i ^ j;
        if (l <= i) continue;
        int up = (i & k) == 0;
        uint64_t x = a[i], y = a[l];
        int swap = up ? (x > y) : (x < y);
        a[i] = swap ? y : x;
        a[l] = swap ? x : y;
      }
  return 0;
}

/* Stages of a shift network over m positions: bits floor(log2(m-1))..0. */
static int or_shift_top(uint64_t m) {
  if (m < 2) return -1;
  int t = 0;
  while ((2ull << t) <= m - 1) ++t;
  return t;
}

#define OR_NONE 0xFFFFFFFFu

/* Expansion: n elements sit at positions 0..n-1; element i must end at
 * target[i], targets strictly increasing and target[i] >= i.  Stage j (from
 * the top bit down) moves an element right by 2^j when bit j of its
 * remaining distance is set.  Each output position reads both candidates
 * (stay / arrive) whatever the data.  out[m] gets payloads, OR_NONE at
 * empty positions.  Returns -1 on a collision (never for valid input). */
int or_expand(const uint32_t* target, const uint32_t* payload, uint64_t n, uint64_t m, uint32_t* out) {
  if (n > m) return -1;
  uint32_t* ct = malloc(m * sizeof(uint32_t));
  uint32_t* cp = malloc(m * sizeof(uint32_t));
  uint32_t* nt = malloc(m * sizeof(uint32_t));
  uint32_t* np = malloc(m * sizeof(uint32_t));
  int rc = 0;
  for (uint64_t p = 0; p < m; ++p) {
    ct[p] = p < n ? target[p] : OR_NONE;
    cp[p] = p < n ? payload[p] : OR_NONE;
  }
  for (int j = or_shift_top(m); j >= 0; --j) {
    uint64_t h = 1ull << j;
#pragma omp parallel for reduction(min : rc) if (m >= 4096)
    for (uint64_t p = 0; p < m; ++p) {
      int stay = ct[p] != OR_NONE && !(((uint64_t)ct[p] - p) & h);
      int arrive = p >= h && ct[p - h] != OR_NONE && ((((uint64_t)ct[p - h] - (p - h)) & h) != 0);
      if (stay && arrive) rc = -1;
      nt[p] = stay ? ct[p] : (arrive ? ct[p - h] : OR_NONE);
      np[p] = stay ? cp[p] : (arrive ? cp[p - h] : OR_NONE);
    }
    uint32_t* t1 = ct; ct = nt; nt = t1;
    uint32_t* t2 = cp; cp = np; np = t2;
  }
  for (uint64_t p = 0; p < m; ++p) {
    if (ct[p] != OR_NONE && ct[p] != p) rc = -1;
    out[p] = cp[p];
  }
  free(ct); free(cp); free(nt); free(np);
  return rc;
}

/* Order-preserving compaction: keep[p] marks the elements to keep; the
 * k-th kept element ends at position k.  Stage j (from bit 0 up) moves an
 * element left by 2^j when bit j of its distance p - k is set.  The inverse
 * of or_expand. */
int or_compact(const uint8_t* keep, const uint32_t* payload, uint64_t m, uint32_t* out) {
  uint32_t* cd = malloc(m * sizeof(uint32_t));
  uint32_t* cp = malloc(m * sizeof(uint32_t));
  uint32_t* nd = malloc(m * sizeof(uint32_t));
  uint32_t* np = malloc(m * sizeof(uint32_t));
  int rc = 0;
  uint64_t k = 0;
  for (uint64_t p = 0; p < m; ++p) {
    cd[p] = keep[p] ? (uint32_t)(p - k) : OR_NONE;
    cp[p] = keep[p] ? payload[p] : OR_NONE;
    k += keep[p] ? 1 : 0;
  }
  int top = or_shift_top(m);
  for (int j = 0; j <= top; ++j) {
    uint64_t h = 1ull << j;
    for (uint64_t p = 0; p < m; ++p) {
      int stay = cd[p] != OR_NONE && !(cd[p] & h);
      int arrive = p + h < m && cd[p + h] != OR_NONE && (cd[p + h] & h);
      if (stay && arrive) rc = -1;
      nd[p] = stay ? cd[p] : (arrive ? cd[p + h] : OR_NONE);
      np[p] = stay ? cp[p] : (arrive ? cp[p + h] : OR_NONE);
    }
    uint32_t* t1 = cd; cd = nd; nd = t1;
    uint32_t* t2 = cp; cp = np; np = t2;
  }
  for (uint64_t p = 0; p < m; ++p) out[p] = cp[p];
  free(cd); free(cp); free(nd); free(np);
  return rc;
}

/* ------------------------------------------------------------------ */
/* 4. The map                                                           */
/* ------------------------------------------------------------------ */

enum { OR_OK = 0, OR_EINVAL = -1, OR_ENOMEM = -2, OR_EDUPKEY = -3, OR_EOVERFLOW = -4, OR_EFULL = -5,
       OR_ESTATE = -7, OR_ETAMPER = -9 /* a sealed page failed its check */,
       OR_EBROKEN = -99 /* internal inconsistency: an oracle bug */ };
enum { OR_GET = 0, OR_PUT = 1, OR_DEL = 2 };
enum { OR_ST_ABSENT = 0, OR_ST_FOUND = 1, OR_ST_UPDATED = 1, OR_ST_INSERTED = 2, OR_ST_DELETED = 3 };

typedef struct { uint32_t batch, kind; uint64_t page; } or_trace_rec; /* kind 0 = read, 1 = write */

typedef struct { uint64_t key; uint32_t p1, p2; } or_pm_entry;

/* A bin decoded from its page bytes. */
typedef struct {
  uint32_t n;
  uint64_t* key; /* Z */
  uint8_t* val;  /* Z * vs */
} or_bin;

typedef struct {
  or_sizes s;
  uint8_t prf_key[32];
  uint8_t* obs;        /* M pages: the observable store */
  uint8_t* hbm;        /* K HBM bins */
  uint32_t* load;      /* B: items in the bin plus stash items destined for it */
  or_pm_entry* rows;   /* R_pm * W */
  uint32_t* rowcnt;    /* R_pm */
  /* eviction stash with a reverse index: one list per bin (Sec. 5.2) */
  uint64_t* st_key;
  uint8_t* st_val;
  uint32_t* st_dest;
  int64_t* st_next;
  int64_t* st_head;    /* B */
  uint64_t st_cap, st_used, st_live;
  uint64_t hbm_live;   /* entries destined for HBM bins (decomposed layout only) */
  int64_t st_free;     /* free list of pool entries */
  /* decomposed HBM store (Sec. 5.2): the items of HBM bins live in the
   * same value pool as the stash, listed under their bin; no HBM pages */
  int decomposed;
  uint64_t ctr, live, batch_no, stash_hw;
  int built, poisoned;
  int trace_on;
  or_trace_rec* trace;
  uint64_t trace_n, trace_cap;
  /* sealing of the observable pages (optional) */
  int seal_on, tampered;
  uint8_t seal_key[32]; /* PRF(domain 4, 0) as 32 bytes */
  uint8_t* tags;        /* M * 16: the pages' Poly1305 tags, observable */
  uint64_t* ver;        /* M: each page's write count, in trusted memory */
} or_map;

static void or_trace_add(or_map* m, uint32_t kind, uint64_t page) {
  if (!m->trace_on) return;
  if (m->trace_n == m->trace_cap) {
    m->trace_cap = m->trace_cap ? 2 * m->trace_cap : 1024;
    m->trace = realloc(m->trace, m->trace_cap * sizeof(or_trace_rec));
  }
  m->trace[m->trace_n].batch = (uint32_t)m->batch_no;
  m->trace[m->trace_n].kind = kind;
  m->trace[m->trace_n].page = page;
  m->trace_n++;
}

/* The nonce of a sealed page: LE32(page index) || LE64(its write count). */
static void or_page_nonce(uint64_t page, uint64_t ver, uint8_t nonce[12]) {
  nonce[0] = (uint8_t)page; nonce[1] = (uint8_t)(page >> 8);
  nonce[2] = (uint8_t)(page >> 16); nonce[3] = (uint8_t)(page >> 24);
  or_put_le64(nonce + 4, ver);
}

/* The only two functions that touch the observable store.  With sealing,
 * a page is written as ChaCha20-Poly1305 of its bytes under the nonce of
 * its next write count, and read back only if its tag checks under the
 * count kept in trusted memory (so a changed, moved or replayed page is
 * refused; the map then fails with OR_ETAMPER). */
static void or_obs_read(or_map* m, uint64_t page, uint8_t* dst) {
  or_trace_add(m, 0, page);
  const uint8_t* src = m->obs + page * m->s.page_bytes;
  if (!m->seal_on) {
    memcpy(dst, src, m->s.page_bytes);
    return;
  }
  uint8_t nonce[12];
  or_page_nonce(page, m->ver[page], nonce);
  if (or_aead_open(m->seal_key, nonce, NULL, 0, src, m->s.page_bytes, m->tags + 16 * page, dst)) {
    m->tampered = 1;
    memset(dst, 0, m->s.page_bytes);
  }
}

static void or_obs_write(or_map* m, uint64_t page, const uint8_t* src) {
  or_trace_add(m, 1, page);
  uint8_t* dst = m->obs + page * m->s.page_bytes;
  if (!m->seal_on) {
    memcpy(dst, src, m->s.page_bytes);
    return;
  }
  uint8_t nonce[12];
  or_page_nonce(page, ++m->ver[page], nonce);
  or_aead_seal(m->seal_key, nonce, NULL, 0, src, m->s.page_bytes, dst, m->tags + 16 * page);
}

/* Turns sealing on (before the build): key = PRF(domain 4, 0). */
int or_set_seal(or_map* m) {
  if (m->built || m->seal_on) return OR_EINVAL;
  uint64_t w[4];
  or_prf(m->prf_key, 4, 0, w);
  for (int j = 0; j < 4; ++j) or_put_le64(m->seal_key + 8 * j, w[j]);
  m->tags = calloc(m->s.M ? m->s.M : 1, 16);
  m->ver = calloc(m->s.M ? m->s.M : 1, sizeof(uint64_t));
  m->seal_on = 1;
  return OR_OK;
}

/* Turns on the decomposed HBM store (before the build): the items of the
 * K HBM bins are kept as value-pool entries listed under their bin (the
 * reverse index the stash already uses), not as dummy-padded pages. */
int or_set_decomposed(or_map* m) {
  if (m->built) return OR_EINVAL;
  m->decomposed = 1;
  return OR_OK;
}

uint8_t* or_tags_ptr(or_map* m) { return m->tags; }
uint64_t* or_ver_ptr(or_map* m) { return m->ver; }

/* What an adversary holding the observable store can do: read or write a
 * page with its tag (page_bytes + 16 bytes), or flip bits of one byte. */
int or_obs_raw(or_map* m, uint64_t page, uint8_t* buf, int write) {
  if (!m->seal_on || page >= m->s.M) return OR_EINVAL;
  uint8_t* pg = m->obs + page * m->s.page_bytes;
  if (write) {
    memcpy(pg, buf, m->s.page_bytes);
    memcpy(m->tags + 16 * page, buf + m->s.page_bytes, 16);
  } else {
    memcpy(buf, pg, m->s.page_bytes);
    memcpy(buf + m->s.page_bytes, m->tags + 16 * page, 16);
  }
  return OR_OK;
}

or_map* or_create(uint64_t cap, uint32_t vs, uint32_t c, uint32_t alpha_pm, uint32_t bin_slots, uint32_t d,
                  uint32_t kpr, uint32_t W, const uint8_t prf_key[32], int trace_on) {
  or_map* m = calloc(1, sizeof(or_map));
  if (!m) return NULL;
  if (or_sizing(cap, vs, c, alpha_pm, bin_slots, d, kpr, W, &m->s)) {
    free(m);
    return NULL;
  }
  memcpy(m->prf_key, prf_key, 32);
  m->obs = calloc(m->s.M ? m->s.M : 1, m->s.page_bytes);
  m->hbm = calloc(m->s.K ? m->s.K : 1, m->s.page_bytes);
  m->load = calloc(m->s.B, sizeof(uint32_t));
  m->rows = calloc(m->s.R_pm * m->s.W, sizeof(or_pm_entry));
  m->rowcnt = calloc(m->s.R_pm, sizeof(uint32_t));
  m->st_head = malloc(m->s.B * sizeof(int64_t));
  for (uint64_t b = 0; b < m->s.B; ++b) m->st_head[b] = -1;
  m->st_free = -1;
  m->trace_on = trace_on;
  return m;
}

void or_destroy(or_map* m) {
  if (!m) return;
  free(m->obs); free(m->hbm); free(m->load); free(m->rows); free(m->rowcnt);
  free(m->st_key); free(m->st_val); free(m->st_dest); free(m->st_next); free(m->st_head);
  free(m->trace);
  free(m->tags); free(m->ver);
  free(m);
}

/* --- pages -------------------------------------------------------- */

static uint8_t* or_page_keys(const or_map* m, uint8_t* page) { (void)m; return page + 8; }
static uint8_t* or_page_vals(const or_map* m, uint8_t* page) { return page + 8 + 8ull * m->s.Z; }

static void or_bin_alloc(const or_map* m, or_bin* b) {
  b->n = 0;
  b->key = malloc(m->s.Z * sizeof(uint64_t));
  b->val = malloc((size_t)m->s.Z * m->s.vs);
}

static void or_bin_free(or_bin* b) { free(b->key); free(b->val); }

static void or_decode(const or_map* m, uint8_t* page, or_bin* b) {
  uint64_t mask = or_le64(page);
  b->n = 0;
  for (uint32_t j = 0; j < m->s.Z; ++j)
    if ((mask >> j) & 1) {
      b->key[b->n] = or_le64(or_page_keys(m, page) + 8 * j);
      memcpy(b->val + (size_t)b->n * m->s.vs, or_page_vals(m, page) + (size_t)j * m->s.vs, m->s.vs);
      b->n++;
    }
}

/* Canonical page: real items first, ascending key; zero everywhere else. */
static void or_encode(const or_map* m, const or_bin* b, uint8_t* page) {
  uint32_t n = b->n, Z = m->s.Z, vs = m->s.vs;
  uint32_t* ord = malloc((n ? n : 1) * sizeof(uint32_t));
  for (uint32_t i = 0; i < n; ++i) ord[i] = i;
  for (uint32_t i = 1; i < n; ++i) /* insertion sort by key */
    for (uint32_t j = i; j > 0 && b->key[ord[j - 1]] > b->key[ord[j]]; --j) {
      uint32_t t = ord[j]; ord[j] = ord[j - 1]; ord[j - 1] = t;
    }
  memset(page, 0, m->s.page_bytes);
  or_put_le64(page, n >= 64 ? ~0ull : ((1ull << n) - 1));
  for (uint32_t i = 0; i < n && i < Z; ++i) {
    or_put_le64(or_page_keys(m, page) + 8 * i, b->key[ord[i]]);
    memcpy(or_page_vals(m, page) + (size_t)i * vs, b->val + (size_t)ord[i] * vs, vs);
  }
  free(ord);
}

/* --- position map (Sec. 5.1 step 3, Sec. 5.2) ---------------------- */

static void or_pm_rows(const or_map* m, uint64_t key, uint64_t rows[8]) {
  uint64_t w[4];
  or_prf(m->prf_key, 2, key, w);
  for (uint32_t j = 0; j < m->s.d; ++j) rows[j] = or_mulhi(w[j], m->s.R_pm);
}

/* Finds key among its d rows; returns 1 and (row, index) on a hit. */
static int or_pm_lookup(const or_map* m, uint64_t key, uint64_t* row, uint32_t* idx) {
  uint64_t rows[8] = {0};
  or_pm_rows(m, key, rows);
  for (uint32_t j = 0; j < m->s.d; ++j) {
    uint64_t r = rows[j];
    for (uint32_t i = 0; i < m->rowcnt[r]; ++i)
      if (m->rows[r * m->s.W + i].key == key) {
        *row = r;
        *idx = i;
        return 1;
      }
  }
  return 0;
}

/* The least-loaded of the d rows, ties to the lowest choice. */
static uint64_t or_pm_choose(const or_map* m, const uint64_t rows[8], const uint32_t* cnt) {
  uint64_t best = rows[0];
  for (uint32_t j = 1; j < m->s.d; ++j)
    if (cnt[rows[j]] < cnt[best]) best = rows[j];
  return best;
}

/* Inserts keys[0..n) with their pairs in rounds of ceil(R_pm/16), each round
 * choosing rows by the counts at its start.  Returns 1 on row overflow. */
static int or_pm_insert_rounds(or_map* m, uint64_t n, const uint64_t* keys, const uint32_t* p1,
                               const uint32_t* p2) {
  uint64_t rs = (m->s.R_pm + 15) / 16;
  uint64_t* choice = malloc((rs ? rs : 1) * sizeof(uint64_t));
  int over = 0;
  for (uint64_t r0 = 0; r0 < n; r0 += rs) {
    uint64_t r1 = r0 + rs < n ? r0 + rs : n;
#pragma omp parallel for
    for (uint64_t i = r0; i < r1; ++i) {
      uint64_t rows[8] = {0};
      or_pm_rows(m, keys[i], rows);
      choice[i - r0] = or_pm_choose(m, rows, m->rowcnt);
    }
    for (uint64_t i = r0; i < r1; ++i) {
      uint64_t r = choice[i - r0];
      if (m->rowcnt[r] >= m->s.W) {
        over = 1;
        continue;
      }
      or_pm_entry* e = &m->rows[r * m->s.W + m->rowcnt[r]];
      e->key = keys[i];
      e->p1 = p1[i];
      e->p2 = p2[i];
      m->rowcnt[r]++;
    }
  }
  free(choice);
  return over;
}

static void or_pm_delete(or_map* m, uint64_t row, uint32_t idx) {
  or_pm_entry* r = &m->rows[row * m->s.W];
  for (uint32_t i = idx + 1; i < m->rowcnt[row]; ++i) r[i - 1] = r[i];
  m->rowcnt[row]--;
}

/* --- stash -------------------------------------------------------- */

static int64_t or_stash_push(or_map* m, uint64_t key, const uint8_t* val, uint32_t dest) {
  int64_t e;
  if (m->st_free >= 0) {
    e = m->st_free;
    m->st_free = m->st_next[e];
  } else {
    if (m->st_used == m->st_cap) {
      m->st_cap = m->st_cap ? 2 * m->st_cap : 1024;
      m->st_key = realloc(m->st_key, m->st_cap * sizeof(uint64_t));
      m->st_val = realloc(m->st_val, m->st_cap * m->s.vs);
      m->st_dest = realloc(m->st_dest, m->st_cap * sizeof(uint32_t));
      m->st_next = realloc(m->st_next, m->st_cap * sizeof(int64_t));
    }
    e = (int64_t)m->st_used++;
  }
  m->st_key[e] = key;
  memcpy(m->st_val + (size_t)e * m->s.vs, val, m->s.vs);
  m->st_dest[e] = dest;
  m->st_next[e] = m->st_head[dest];
  m->st_head[dest] = e;
  m->st_live++;
  if (dest < m->s.K) m->hbm_live++;
  return e;
}

/* Unlinks entry e from the list of its bin and frees it. */
static void or_stash_remove(or_map* m, int64_t e) {
  uint32_t b = m->st_dest[e];
  int64_t* pp = &m->st_head[b];
  while (*pp != e) pp = &m->st_next[*pp];
  *pp = m->st_next[e];
  m->st_next[e] = m->st_free;
  m->st_free = e;
  m->st_live--;
  if (b < m->s.K) m->hbm_live--;
}

/* --- build -------------------------------------------------------- */

/* mode 0: the oblivious procedure (PRF, P2C rounds, bitonic sort of
 *         (bin, index) tags, rank, expansion network, page write-out).
 * mode 1: the plain definition of the same result: each bin holds the keys
 *         whose P2C choice it is, written as a canonical page.
 * Both end in the same state; the tests check that. */
int or_build(or_map* m, const uint64_t* keys, const uint8_t* vals, uint64_t n, int mode) {
  if (m->poisoned) return OR_ESTATE;
  if (m->built || n > m->s.cap) return OR_EINVAL;
  const or_sizes* s = &m->s;
  uint32_t* p1 = malloc((n ? n : 1) * sizeof(uint32_t));
  uint32_t* p2 = malloc((n ? n : 1) * sizeof(uint32_t));
  uint32_t* dest = malloc((n ? n : 1) * sizeof(uint32_t));
  int over = 0;

  /* a1: two distinct random bins per key (Sec. 4.1: "each data item is
   * initially assigned to two uniformly chosen random bins"). */
#pragma omp parallel for
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t w[4];
    or_prf(m->prf_key, 1, keys[i], w);
    or_pair(w[0], w[1], s->B, &p1[i], &p2[i]);
  }
  /* a2: P2C placement, in rounds that see the loads at their start. */
  uint64_t rs = (s->B + 15) / 16;
  for (uint64_t r0 = 0; r0 < n; r0 += rs) {
    uint64_t r1 = r0 + rs < n ? r0 + rs : n;
#pragma omp parallel for
    for (uint64_t i = r0; i < r1; ++i) dest[i] = m->load[p2[i]] < m->load[p1[i]] ? p2[i] : p1[i];
    for (uint64_t i = r0; i < r1; ++i) m->load[dest[i]]++;
  }
  for (uint64_t b = 0; b < s->B; ++b)
    if (m->load[b] > s->Z) over = 1;

  uint8_t* page = malloc(s->page_bytes);
  or_bin bin;
  or_bin_alloc(m, &bin);
  m->batch_no = 0;
  if (!over) {
    uint64_t BZ = s->B * s->Z;
    uint32_t* slot_src = malloc(BZ * sizeof(uint32_t));
    if (mode == 0) {
      /* a3: bitonic sort of tags (bin << 32 | input index), padded to a
       * power of two with tags of bin 0xFFFFFFFF. */
      uint64_t np2 = 1;
      while (np2 < n) np2 <<= 1;
      uint64_t* tag = malloc(np2 * sizeof(uint64_t));
      for (uint64_t i = 0; i < np2; ++i)
        tag[i] = i < n ? (((uint64_t)dest[i] << 32) | i) : ((0xFFFFFFFFull << 32) | i);
      or_bitonic_sort_u64(tag, np2);
      /* a4: rank inside the run of equal bins; target slot bin * Z + rank. */
      uint32_t* tgt = malloc((n ? n : 1) * sizeof(uint32_t));
      uint32_t* src = malloc((n ? n : 1) * sizeof(uint32_t));
      uint32_t rank = 0;
      for (uint64_t i = 0; i < n; ++i) {
        uint32_t b = (uint32_t)(tag[i] >> 32);
        rank = (i > 0 && (uint32_t)(tag[i - 1] >> 32) == b) ? rank + 1 : 0;
        tgt[i] = (uint32_t)(b * (uint64_t)s->Z + rank);
        src[i] = (uint32_t)tag[i];
      }
      /* a5: expansion network into B * Z slots. */
      if (BZ >= 2) {
        if (or_expand(tgt, src, n, BZ, slot_src)) over = 1;
      } else {
        slot_src[0] = n ? src[0] : OR_NONE;
      }
      free(tag); free(tgt); free(src);
    } else {
      /* plain definition: each bin lists its keys in input order */
      uint32_t* fill = calloc(s->B, sizeof(uint32_t));
      for (uint64_t p = 0; p < BZ; ++p) slot_src[p] = OR_NONE;
      for (uint64_t i = 0; i < n; ++i) slot_src[(uint64_t)dest[i] * s->Z + fill[dest[i]]++] = (uint32_t)i;
      free(fill);
    }
    /* a6: write every bin as a canonical page: HBM bins, then observable
     * pages 0..M-1 in order (in parallel only when no trace is kept). */
#pragma omp parallel if (!m->trace_on)
    {
      or_bin wbin;
      or_bin_alloc(m, &wbin);
      uint8_t* wpage = malloc(s->page_bytes);
#pragma omp for
      for (uint64_t b = 0; b < s->B; ++b) {
        wbin.n = 0;
        for (uint32_t j = 0; j < s->Z; ++j) {
          uint32_t i = slot_src[b * s->Z + j];
          if (i == OR_NONE) continue;
          wbin.key[wbin.n] = keys[i];
          memcpy(wbin.val + (size_t)wbin.n * s->vs, vals + (size_t)i * s->vs, s->vs);
          wbin.n++;
        }
        if (b < s->K && m->decomposed) continue; /* pushed to the value pool below */
        or_encode(m, &wbin, wpage);
        if (b < s->K)
          memcpy(m->hbm + b * s->page_bytes, wpage, s->page_bytes);
        else
          or_obs_write(m, b - s->K, wpage);
      }
      or_bin_free(&wbin);
      free(wpage);
    }
    if (m->decomposed) /* the HBM bins' items into the value pool, bin by bin */
      for (uint64_t b = 0; b < s->K; ++b)
        for (uint32_t j = 0; j < s->Z; ++j) {
          uint32_t i = slot_src[b * s->Z + j];
          if (i != OR_NONE) or_stash_push(m, keys[i], vals + (size_t)i * s->vs, (uint32_t)b);
        }
    if (m->hbm_live > s->hbm_bound) over = 1;
    free(slot_src);
    /* a7: position map (key -> p1, p2), d-choice rows in rounds. */
    if (or_pm_insert_rounds(m, n, keys, p1, p2)) over = 1;
  }
  int rc = OR_OK;
  if (over) {
    rc = OR_EOVERFLOW;
  } else {
    /* duplicate keys: a key found more than once among its rows */
    int dup = 0;
#pragma omp parallel for reduction(| : dup)
    for (uint64_t i = 0; i < n; ++i) {
      uint64_t rows[8] = {0};
      or_pm_rows(m, keys[i], rows);
      uint32_t hits = 0;
      for (uint32_t j = 0; j < s->d; ++j) {
        int seen = 0;
        for (uint32_t jj = 0; jj < j; ++jj) seen |= rows[jj] == rows[j];
        if (seen) continue;
        for (uint32_t e = 0; e < m->rowcnt[rows[j]]; ++e) hits += m->rows[rows[j] * s->W + e].key == keys[i];
      }
      dup |= hits > 1;
    }
    if (dup) rc = OR_EDUPKEY;
  }
  or_bin_free(&bin);
  free(page); free(p1); free(p2); free(dest);
  if (rc) {
    m->poisoned = 1;
    return rc;
  }
  m->built = 1;
  m->live = n;
  m->ctr = 0;
  return OR_OK;
}

/* --- batched access (Alg. 1; Sec. 5.1 steps 2-6) ------------------- */

typedef struct { uint64_t key; uint32_t idx; } or_kidx;

static int or_cmp_kidx(const void* a, const void* b) {
  const or_kidx* x = a;
  const or_kidx* y = b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  return x->idx < y->idx ? -1 : (x->idx > y->idx);
}

static int or_cmp_u64(const void* a, const void* b) {
  uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
  return x < y ? -1 : (x > y);
}

/* The working copy of a bin touched in this batch. */
typedef struct {
  int64_t* slot;   /* B: index into work[], -1 if untouched */
  or_bin* work;
  uint64_t* bin_of;
  uint64_t n, cap;
} or_workset;

static or_bin* or_work_get(or_map* m, or_workset* w, uint64_t b, const uint8_t* page_if_new) {
  if (w->slot[b] >= 0) return &w->work[w->slot[b]];
  if (w->n == w->cap) {
    w->cap = w->cap ? 2 * w->cap : 64;
    w->work = realloc(w->work, w->cap * sizeof(or_bin));
    w->bin_of = realloc(w->bin_of, w->cap * sizeof(uint64_t));
  }
  or_bin* x = &w->work[w->n];
  or_bin_alloc(m, x);
  or_decode(m, (uint8_t*)page_if_new, x);
  w->bin_of[w->n] = b;
  w->slot[b] = (int64_t)w->n;
  w->n++;
  return x;
}

/* Removes key from bin b (its page or HBM slots, or the stash list of b).
 * Returns 1 and copies the value out if found. */
static int or_find_remove(or_map* m, or_bin* wb, uint64_t b, uint64_t key, uint8_t* val) {
  for (uint32_t i = 0; i < wb->n; ++i)
    if (wb->key[i] == key) {
      memcpy(val, wb->val + (size_t)i * m->s.vs, m->s.vs);
      for (uint32_t j = i + 1; j < wb->n; ++j) {
        wb->key[j - 1] = wb->key[j];
        memcpy(wb->val + (size_t)(j - 1) * m->s.vs, wb->val + (size_t)j * m->s.vs, m->s.vs);
      }
      wb->n--;
      return 1;
    }
  for (int64_t e = m->st_head[b]; e >= 0; e = m->st_next[e])
    if (m->st_key[e] == key) {
      memcpy(val, m->st_val + (size_t)e * m->s.vs, m->s.vs);
      or_stash_remove(m, e);
      return 1;
    }
  return 0;
}

int or_access(or_map* m, const uint8_t* ops, const uint64_t* keys, const uint8_t* vals_in, uint8_t* vals_out,
              uint8_t* status, uint32_t q) {
  if (m->poisoned) return OR_ESTATE;
  if (!m->built) return OR_EINVAL;
  if (q == 0) return OR_OK;
  /* a batch with a bad op code keeps its number (as a label of the trace)
     but changes nothing and records no access */
  m->batch_no++;
  for (uint32_t i = 0; i < q; ++i)
    if (ops[i] > OR_DEL) return OR_EINVAL;
  const or_sizes* s = &m->s;
  uint32_t vs = s->vs;

  /* leaders: the first occurrence of each key, found by sorting (key, i) */
  or_kidx* kx = malloc(q * sizeof(or_kidx));
  for (uint32_t i = 0; i < q; ++i) {
    kx[i].key = keys[i];
    kx[i].idx = i;
  }
  qsort(kx, q, sizeof(or_kidx), or_cmp_kidx);
  uint32_t* leader = malloc(q * sizeof(uint32_t));
  for (uint32_t r = 0; r < q; ++r)
    leader[kx[r].idx] = (r > 0 && kx[r - 1].key == kx[r].key) ? leader[kx[r - 1].idx] : kx[r].idx;

  /* per-leader in-flight state */
  uint8_t* hit = calloc(q, 1);
  uint8_t* present = calloc(q, 1);
  uint8_t* cur = calloc((size_t)q * vs, 1);
  uint64_t* hrow = calloc(q, sizeof(uint64_t));
  uint32_t* hidx = calloc(q, sizeof(uint32_t));
  uint32_t* r1 = calloc(q, sizeof(uint32_t));
  uint32_t* r2 = calloc(q, sizeof(uint32_t));
  uint64_t* fetched = malloc(2ull * q * sizeof(uint64_t));
  uint64_t nfetched = 0;
  or_workset ws = {0};
  ws.slot = malloc(s->B * sizeof(int64_t));
  for (uint64_t b = 0; b < s->B; ++b) ws.slot[b] = -1;
  uint8_t* page = malloc(s->page_bytes);
  int broken = 0;

  /* Each command's tape pairs, and each leader's position-map entry (the
   * map does not change until every command has run). */
  uint32_t* f1 = malloc(q * sizeof(uint32_t));
  uint32_t* f2 = malloc(q * sizeof(uint32_t));
#pragma omp parallel for
  for (uint32_t i = 0; i < q; ++i) {
    uint64_t w[4];
    or_prf(m->prf_key, 3, m->ctr + i, w);
    or_pair(w[0], w[1], s->B, &f1[i], &f2[i]);  /* F(s): pair for dummy reads */
    or_pair(w[2], w[3], s->B, &r1[i], &r2[i]); /* R(s): new pair on remap */
    if (leader[i] == i) hit[i] = (uint8_t)or_pm_lookup(m, keys[i], &hrow[i], &hidx[i]);
  }

  /* Steps 2-4 and 6 of Sec. 5.1, one command at a time. */
  for (uint32_t i = 0; i < q; ++i) {
    uint64_t k = keys[i];
    uint32_t pr[2] = {f1[i], f2[i]};
    if (hit[i]) {
      pr[0] = m->rows[hrow[i] * s->W + hidx[i]].p1;
      pr[1] = m->rows[hrow[i] * s->W + hidx[i]].p2;
    }
    /* Alg. 1, the loop over (p1, p2): read both bins. */
    for (int role = 0; role < 2; ++role) {
      uint64_t b = pr[role];
      or_bin* wb;
      if (b >= s->K) {
        or_obs_read(m, b - s->K, page);
        fetched[nfetched++] = b - s->K;
        wb = or_work_get(m, &ws, b, page);
      } else {
        wb = or_work_get(m, &ws, b, m->hbm + b * s->page_bytes);
      }
      if (hit[i] && !present[i] && or_find_remove(m, wb, b, k, cur + (size_t)i * vs)) {
        present[i] = 1;
        m->load[b]--;
      }
    }
    if (hit[i] && !present[i]) broken = 1; /* a mapped key must sit in one of its bins */
    /* exec_cmd on the key's current state */
    uint32_t L = leader[i];
    uint8_t* vo = vals_out + (size_t)i * vs;
    memset(vo, 0, vs);
    if (ops[i] == OR_GET) {
      status[i] = present[L] ? OR_ST_FOUND : OR_ST_ABSENT;
      if (present[L]) memcpy(vo, cur + (size_t)L * vs, vs);
    } else if (ops[i] == OR_PUT) {
      status[i] = present[L] ? OR_ST_UPDATED : OR_ST_INSERTED;
      present[L] = 1;
      memcpy(cur + (size_t)L * vs, vals_in + (size_t)i * vs, vs);
    } else {
      status[i] = present[L] ? OR_ST_DELETED : OR_ST_ABSENT;
      present[L] = 0;
    }
  }

  /* Step 5 of Sec. 5.1 (random_remap + P2C_load_balance of Alg. 1), for each
   * key present at the end, in rounds over the post-removal loads. */
  int over = 0;
  uint64_t rs = (s->B + 15) / 16;
  uint32_t* ord = malloc(q * sizeof(uint32_t));
  uint32_t* chosen = malloc(q * sizeof(uint32_t));
  uint32_t nplace = 0;
  for (uint32_t i = 0; i < q; ++i)
    if (leader[i] == i && present[i]) ord[nplace++] = i;
  for (uint64_t o0 = 0; o0 < nplace; o0 += rs) {
    uint64_t o1 = o0 + rs < nplace ? o0 + rs : nplace;
#pragma omp parallel for
    for (uint64_t o = o0; o < o1; ++o) {
      uint32_t i = ord[o];
      chosen[o] = m->load[r2[i]] < m->load[r1[i]] ? r2[i] : r1[i];
    }
    for (uint64_t o = o0; o < o1; ++o) m->load[chosen[o]]++;
  }
  for (uint32_t o = 0; o < nplace; ++o)
    if (m->load[chosen[o]] > s->Z) over = 1;
  if (!over)
    for (uint32_t o = 0; o < nplace; ++o) {
      uint32_t i = ord[o];
      uint64_t b = chosen[o];
      if (b < s->K && !m->decomposed) { /* HBM bin: insert directly */
        or_bin* wb = or_work_get(m, &ws, b, m->hbm + b * s->page_bytes);
        wb->key[wb->n] = keys[i];
        memcpy(wb->val + (size_t)wb->n * vs, cur + (size_t)i * vs, vs);
        wb->n++;
      } else { /* host bin (or any bin of a decomposed store): into the value pool */
        or_stash_push(m, keys[i], cur + (size_t)i * vs, (uint32_t)b);
      }
    }

  /* position map: new pairs for hits that stay, deletes, then inserts */
  uint64_t ndel = 0, nins = 0;
  uint64_t* ins_key = malloc(q * sizeof(uint64_t));
  uint32_t* ins_p1 = malloc(q * sizeof(uint32_t));
  uint32_t* ins_p2 = malloc(q * sizeof(uint32_t));
  if (!over) {
    for (uint32_t i = 0; i < q; ++i) {
      if (leader[i] != i || !hit[i] || !present[i]) continue;
      or_pm_entry* e = &m->rows[hrow[i] * s->W + hidx[i]];
      e->p1 = r1[i];
      e->p2 = r2[i];
    }
    /* deletes in descending (row, index) so earlier indexes stay valid */
    uint64_t* del = malloc(q * sizeof(uint64_t));
    for (uint32_t i = 0; i < q; ++i)
      if (leader[i] == i && hit[i] && !present[i]) del[ndel++] = (hrow[i] << 32) | hidx[i];
    qsort(del, ndel, sizeof(uint64_t), or_cmp_u64);
    for (uint64_t x = ndel; x-- > 0;) or_pm_delete(m, del[x] >> 32, (uint32_t)del[x]);
    free(del);
    for (uint32_t i = 0; i < q; ++i) {
      if (leader[i] != i || hit[i] || !present[i]) continue;
      ins_key[nins] = keys[i];
      ins_p1[nins] = r1[i];
      ins_p2[nins] = r2[i];
      nins++;
    }
    if (or_pm_insert_rounds(m, nins, ins_key, ins_p1, ins_p2)) over = 1;
  }

  /* write-back with eviction: each distinct page read, ascending */
  if (!over) {
    qsort(fetched, nfetched, sizeof(uint64_t), or_cmp_u64);
    for (uint64_t f = 0; f < nfetched; ++f) {
      if (f > 0 && fetched[f] == fetched[f - 1]) continue;
      uint64_t b = fetched[f] + s->K;
      or_bin* wb = &ws.work[ws.slot[b]];
      while (m->st_head[b] >= 0) { /* evict everything destined here */
        int64_t e = m->st_head[b];
        wb->key[wb->n] = m->st_key[e];
        memcpy(wb->val + (size_t)wb->n * vs, m->st_val + (size_t)e * vs, vs);
        wb->n++;
        or_stash_remove(m, e);
      }
      or_encode(m, wb, page);
      or_obs_write(m, fetched[f], page);
    }
    for (uint64_t x = 0; x < ws.n; ++x) /* HBM bins: no observable access */
      if (ws.bin_of[x] < s->K && !m->decomposed) or_encode(m, &ws.work[x], m->hbm + ws.bin_of[x] * s->page_bytes);
    uint64_t host_live = m->st_live - m->hbm_live; /* the stash proper: items bound for host pages */
    if (host_live > s->stash_bound) over = 1;
    if (m->hbm_live > s->hbm_bound) over = 1;
    if (host_live > m->stash_hw) m->stash_hw = host_live;
  }

  for (uint64_t x = 0; x < ws.n; ++x) or_bin_free(&ws.work[x]);
  free(ws.work); free(ws.bin_of); free(ws.slot);
  free(kx); free(leader); free(hit); free(present); free(cur); free(hrow); free(hidx);
  free(r1); free(r2); free(f1); free(f2); free(fetched); free(page); free(ord); free(chosen);
  free(ins_key); free(ins_p1); free(ins_p2);
  m->ctr += q;
  if (m->tampered) {
    m->poisoned = 1;
    return OR_ETAMPER;
  }
  if (broken) {
    m->poisoned = 1;
    return OR_EBROKEN;
  }
  if (over) {
    m->poisoned = 1;
    return OR_EOVERFLOW;
  }
  m->live = m->live + nins - ndel;
  if (m->live > s->cap) {
    m->poisoned = 1;
    return OR_EFULL;
  }
  return OR_OK;
}

/* ------------------------------------------------------------------ */
/* 5. The plain definition of the answers (O1), in C                    */
/* ------------------------------------------------------------------ */

/* A non-oblivious dictionary with the Get / Put / Delete semantics of
 * Sec. 2.1 (delete = a tombstone put): an open-addressing hash table with
 * linear probing and backward-shift deletion.  It gives the same answers
 * as the Python dictionary of oracle/__init__.py (the tests check that)
 * and serves as the timed plain baseline. */
typedef struct {
  uint64_t mask, n;
  uint32_t vs;
  uint64_t* key;
  uint8_t* used;
  uint8_t* val;
} or_plain;

static uint64_t or_plain_hash(uint64_t k) { /* SplitMix64 finalizer */
  k ^= k >> 30;
  k *= 0xBF58476D1CE4E5B9ull;
  k ^= k >> 27;
  k *= 0x94D049BB133111EBull;
  return k ^ (k >> 31);
}

or_plain* or_plain_create(uint64_t cap, uint32_t vs) {
  or_plain* p = calloc(1, sizeof(or_plain));
  if (!p) return NULL;
  uint64_t size = 16;
  while (size < 2 * cap + 2) size <<= 1;
  p->mask = size - 1;
  p->vs = vs;
  p->key = calloc(size, sizeof(uint64_t));
  p->used = calloc(size, 1);
  p->val = calloc(size, vs);
  if (!p->key || !p->used || !p->val) {
    free(p->key); free(p->used); free(p->val); free(p);
    return NULL;
  }
  return p;
}

void or_plain_destroy(or_plain* p) {
  if (!p) return;
  free(p->key); free(p->used); free(p->val); free(p);
}

/* The slot holding k, or the empty slot where it would go. */
static uint64_t or_plain_slot(const or_plain* p, uint64_t k) {
  uint64_t i = or_plain_hash(k) & p->mask;
  while (p->used[i] && p->key[i] != k) i = (i + 1) & p->mask;
  return i;
}

static void or_plain_erase(or_plain* p, uint64_t i) {
  p->used[i] = 0;
  p->n--;
  uint64_t j = i;
  for (;;) { /* shift back later members of the cluster that may fill the hole */
    j = (j + 1) & p->mask;
    if (!p->used[j]) return;
    uint64_t h = or_plain_hash(p->key[j]) & p->mask;
    /* j's entry may move to i when its home h is not cyclically in (i, j] */
    int in_range = i <= j ? (h > i && h <= j) : (h > i || h <= j);
    if (in_range) continue;
    p->key[i] = p->key[j];
    memcpy(p->val + i * p->vs, p->val + j * p->vs, p->vs);
    p->used[i] = 1;
    p->used[j] = 0;
    i = j;
  }
}

/* Inserts (returns 0) or refuses when the table is at its capacity (-1). */
static int or_plain_put(or_plain* p, uint64_t k, const uint8_t* v, int* inserted) {
  uint64_t i = or_plain_slot(p, k);
  *inserted = !p->used[i];
  if (*inserted) {
    if (2 * (p->n + 1) > p->mask + 1) return -1;
    p->used[i] = 1;
    p->key[i] = k;
    p->n++;
  }
  memcpy(p->val + i * p->vs, v, p->vs);
  return 0;
}

int or_plain_build(or_plain* p, const uint64_t* keys, const uint8_t* vals, uint64_t n) {
  for (uint64_t i = 0; i < n; ++i) {
    int ins;
    if (or_plain_put(p, keys[i], vals + i * p->vs, &ins)) return OR_EFULL;
    if (!ins) return OR_EDUPKEY;
  }
  return OR_OK;
}

/* The commands in order: GET answers (found, value) or (absent, zeros);
 * PUT answers updated or inserted; DEL answers deleted or absent. */
int or_plain_access(or_plain* p, const uint8_t* ops, const uint64_t* keys, const uint8_t* vals_in, uint8_t* vals_out,
                    uint8_t* status, uint32_t q) {
  for (uint32_t i = 0; i < q; ++i)
    if (ops[i] > OR_DEL) return OR_EINVAL;
  for (uint32_t i = 0; i < q; ++i) {
    uint64_t s = or_plain_slot(p, keys[i]);
    int had = p->used[s];
    uint8_t* vo = vals_out + (size_t)i * p->vs;
    memset(vo, 0, p->vs);
    if (ops[i] == OR_GET) {
      status[i] = had ? OR_ST_FOUND : OR_ST_ABSENT;
      if (had) memcpy(vo, p->val + s * p->vs, p->vs);
    } else if (ops[i] == OR_PUT) {
      int ins;
      if (or_plain_put(p, keys[i], vals_in + (size_t)i * p->vs, &ins)) return OR_EFULL;
      status[i] = ins ? OR_ST_INSERTED : OR_ST_UPDATED;
    } else {
      status[i] = had ? OR_ST_DELETED : OR_ST_ABSENT;
      if (had) or_plain_erase(p, s);
    }
  }
  return OR_OK;
}

uint64_t or_plain_size(const or_plain* p) { return p->n; }

/* --- state readout (tests) ---------------------------------------- */

const or_sizes* or_get_sizes(const or_map* m) { return &m->s; }
const uint8_t* or_obs_ptr(const or_map* m) { return m->obs; }
const uint8_t* or_hbm_ptr(const or_map* m) { return m->hbm; }
const uint32_t* or_load_ptr(const or_map* m) { return m->load; }
uint64_t or_ctr(const or_map* m) { return m->ctr; }
uint64_t or_live(const or_map* m) { return m->live; }
uint64_t or_stash_live(const or_map* m) { return m->st_live - m->hbm_live; }
uint64_t or_hbm_live(const or_map* m) { return m->hbm_live; }
uint64_t or_stash_highwater(const or_map* m) { return m->stash_hw; }
uint64_t or_trace_len(const or_map* m) { return m->trace_n; }

uint64_t or_trace_copy(const or_map* m, or_trace_rec* out, uint64_t cap) {
  uint64_t n = m->trace_n < cap ? m->trace_n : cap;
  memcpy(out, m->trace, n * sizeof(or_trace_rec));
  return n;
}

void or_trace_clear(or_map* m) { m->trace_n = 0; }

/* Stash entries as (key, dest bin) plus values; returns the count. */
uint64_t or_stash_copy(const or_map* m, uint64_t* key, uint32_t* dest, uint8_t* val, uint64_t cap) {
  uint64_t n = 0;
  for (uint64_t b = 0; b < m->s.B; ++b)
    for (int64_t e = m->st_head[b]; e >= 0; e = m->st_next[e]) {
      if (n < cap) {
        key[n] = m->st_key[e];
        dest[n] = m->st_dest[e];
        memcpy(val + n * m->s.vs, m->st_val + (size_t)e * m->s.vs, m->s.vs);
      }
      n++;
    }
  return n;
}

/* Position map as (row, key, p1, p2); returns the count. */
uint64_t or_pm_copy(const or_map* m, uint64_t* row, uint64_t* key, uint32_t* p1, uint32_t* p2, uint64_t cap) {
  uint64_t n = 0;
  for (uint64_t r = 0; r < m->s.R_pm; ++r)
    for (uint32_t i = 0; i < m->rowcnt[r]; ++i) {
      if (n < cap) {
        const or_pm_entry* e = &m->rows[r * m->s.W + i];
        row[n] = r;
        key[n] = e->key;
        p1[n] = e->p1;
        p2[n] = e->p2;
      }
      n++;
    }
  return n;
}

uint32_t or_pm_max_row(const or_map* m) {
  uint32_t mx = 0;
  for (uint64_t r = 0; r < m->s.R_pm; ++r)
    if (m->rowcnt[r] > mx) mx = m->rowcnt[r];
  return mx;
}
