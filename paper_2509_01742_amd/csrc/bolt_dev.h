// Device-side building blocks of the oblivious map: the keyed PRF, range
// reduction to bins, and the layout of the control block every kernel
// shares.  Written for gfx950 (wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bolt {

constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint64_t kNone64 = 0xFFFFFFFFFFFFFFFFull;
constexpr uint32_t kMaxBatch = 8192;
constexpr uint32_t kWave = 64;

// Sticky error bits kept on the device (host maps them to return codes).
constexpr uint32_t kErrOverflow = 1u;  // bin, stash or row capacity
constexpr uint32_t kErrFull = 2u;      // live keys beyond capacity
constexpr uint32_t kErrDup = 4u;       // duplicate build keys
constexpr uint32_t kErrBroken = 8u;    // internal inconsistency (a library bug)
constexpr uint32_t kErrTrace = 16u;    // trace log full (not sticky for the map)
constexpr uint32_t kErrTamper = 32u;   // a sealed page failed its check

// State that kernels of one map read and update on the device.
struct Ctl {
  uint32_t hkey[8];      // BLAKE2s chaining value after the padded key block
  uint32_t skey[8];      // page-sealing key: PRF(domain 4, 0) as eight LE words
  uint32_t err;          // sticky error bits
  uint32_t reject;       // current batch rejected (bad op code)
  uint64_t steps;        // tape counter s
  uint64_t live;         // keys present
  uint64_t stash_live;   // stash pool entries in use at the end of the last batch
  uint64_t stash_hw;     // stash high-water mark
  uint32_t b_place;      // items placed by the current batch
  uint32_t b_ins;        // keys inserted by the current batch
  uint32_t b_del;        // keys deleted by the current batch
  uint32_t load_hw;      // BOLT_F_WATCH: largest bin load seen at a batch end
  uint64_t hbm_load;     // BOLT_F_WATCH: items in the HBM bins at the last batch end
  uint64_t hbm_hw;       // BOLT_F_WATCH: largest hbm_load seen
  uint32_t ckey[8];      // BOLT_F_SEAL_CMDS: session key of the command and response records
  uint64_t seq;          // BOLT_F_SEAL_CMDS: sealed requests run so far (the next is seq + 1)
  // BOLT_F_DECOMPOSED: the free-address ring of the value pool and the
  // pool's HBM-bin items.  Ring positions [ring_head, ring_tail) hold the
  // free entries (modulo the pool size); a batch takes ring_take of them
  // from the head and returns ring_give at the tail, both folded in at its
  // end.
  uint64_t ring_head, ring_tail;
  uint32_t ring_take, ring_give;
  uint64_t pool_live;    // pool entries in use at the end of the last batch (stash plus HBM-bin items)
  uint64_t hbm_live;     // of which items of HBM bins
  uint32_t b_hbm_in;     // items the current batch placed in HBM bins
  uint32_t b_hbm_rm;     // items the current batch removed from HBM bins
  uint32_t fin_done;     // BOLT_F_DECOMPOSED: finish workgroups done with their share of the ring returns
  uint32_t pad0;
};

// ---------------------------------------------------------------------------
// BLAKE2s (RFC 7693).  Keyed PRF on a nine-byte message (domain, LE64(x)):
// with a 32-byte key the key block is the same for every message, so it is
// compressed once per map (prf_key_setup) and each PRF call is the one final
// compression of the message block with counter 64 + 9.
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t rotr32(uint32_t x, int n) { return __builtin_rotateright32(x, n); }

struct B2sIv {
  static constexpr uint32_t v[8] = {0x6A09E667u, 0xBB67AE85u, 0x3C6EF372u, 0xA54FF53Au,
                                    0x510E527Fu, 0x9B05688Cu, 0x1F83D9ABu, 0x5BE0CD19u};
};

// Message schedule of the ten rounds (RFC 7693, Sec. 2.7).
constexpr uint8_t kSigma[10][16] = {
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

#define BOLT_B2S_G(a, b, c, d, x, y) \
  do {                               \
    a = a + b + (x);                 \
    d = rotr32(d ^ a, 16);           \
    c = c + d;                       \
    b = rotr32(b ^ c, 12);           \
    a = a + b + (y);                 \
    d = rotr32(d ^ a, 8);            \
    c = c + d;                       \
    b = rotr32(b ^ c, 7);            \
  } while (0)

// One compression of block m[16] into h[8] with byte counter t.
__device__ __forceinline__ void b2s_compress(uint32_t h[8], const uint32_t m[16], uint32_t t, bool last) {
  uint32_t v0 = h[0], v1 = h[1], v2 = h[2], v3 = h[3], v4 = h[4], v5 = h[5], v6 = h[6], v7 = h[7];
  uint32_t v8 = B2sIv::v[0], v9 = B2sIv::v[1], v10 = B2sIv::v[2], v11 = B2sIv::v[3];
  uint32_t v12 = B2sIv::v[4] ^ t, v13 = B2sIv::v[5], v14 = last ? ~B2sIv::v[6] : B2sIv::v[6], v15 = B2sIv::v[7];
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    BOLT_B2S_G(v0, v4, v8, v12, m[kSigma[r][0]], m[kSigma[r][1]]);
    BOLT_B2S_G(v1, v5, v9, v13, m[kSigma[r][2]], m[kSigma[r][3]]);
    BOLT_B2S_G(v2, v6, v10, v14, m[kSigma[r][4]], m[kSigma[r][5]]);
    BOLT_B2S_G(v3, v7, v11, v15, m[kSigma[r][6]], m[kSigma[r][7]]);
    BOLT_B2S_G(v0, v5, v10, v15, m[kSigma[r][8]], m[kSigma[r][9]]);
    BOLT_B2S_G(v1, v6, v11, v12, m[kSigma[r][10]], m[kSigma[r][11]]);
    BOLT_B2S_G(v2, v7, v8, v13, m[kSigma[r][12]], m[kSigma[r][13]]);
    BOLT_B2S_G(v3, v4, v9, v14, m[kSigma[r][14]], m[kSigma[r][15]]);
  }
  h[0] ^= v0 ^ v8;
  h[1] ^= v1 ^ v9;
  h[2] ^= v2 ^ v10;
  h[3] ^= v3 ^ v11;
  h[4] ^= v4 ^ v12;
  h[5] ^= v5 ^ v13;
  h[6] ^= v6 ^ v14;
  h[7] ^= v7 ^ v15;
}

// Chaining value after the first block (the 32-byte key padded to 64 bytes)
// of BLAKE2s-256 with a 32-byte key.
__device__ inline void b2s_key_block(const uint32_t key_words[8], uint32_t h[8]) {
#pragma unroll
  for (int i = 0; i < 8; ++i) h[i] = B2sIv::v[i];
  h[0] ^= 0x01010000u ^ (32u << 8) ^ 32u;
  uint32_t m[16];
#pragma unroll
  for (int i = 0; i < 8; ++i) m[i] = key_words[i];
#pragma unroll
  for (int i = 8; i < 16; ++i) m[i] = 0;
  b2s_compress(h, m, 64, false);
}

// PRF(domain, x) -> w[0..3], the digest as little-endian 64-bit words.
__device__ __forceinline__ void prf4(const uint32_t hkey[8], uint32_t domain, uint64_t x, uint64_t w[4]) {
  uint32_t m[16];
  m[0] = domain | ((uint32_t)x << 8);      // bytes 0..3: domain, x0..x2
  m[1] = (uint32_t)(x >> 24);              // bytes 4..7: x3..x6
  m[2] = (uint32_t)(x >> 56);              // byte 8: x7
#pragma unroll
  for (int i = 3; i < 16; ++i) m[i] = 0;
  uint32_t h[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) h[i] = hkey[i];
  b2s_compress(h, m, 64 + 9, true);
#pragma unroll
  for (int j = 0; j < 4; ++j) w[j] = (uint64_t)h[2 * j] | ((uint64_t)h[2 * j + 1] << 32);
}

// Two distinct bins in [0, B) from two PRF words (uniform over the B(B-1)
// ordered pairs, up to a bias below B / 2^64).
__device__ __forceinline__ void pair_of(uint64_t w0, uint64_t w1, uint64_t B, uint32_t& p1, uint32_t& p2) {
  uint64_t a = __umul64hi(w0, B);
  uint64_t b = a + 1 + __umul64hi(w1, B - 1);
  if (b >= B) b -= B;
  p1 = (uint32_t)a;
  p2 = (uint32_t)b;
}

// Domains of the PRF input.
constexpr uint32_t kDomPair = 1;  // a key's two bins at build time
constexpr uint32_t kDomRows = 2;  // a key's position-map rows
constexpr uint32_t kDomTape = 3;  // step s: fetch pair F(s) and remap pair R(s)
constexpr uint32_t kDomSeal = 4;  // x = 0: the key that seals observable pages

// ---------------------------------------------------------------------------
// Small helpers.
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint64_t ld_acq64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_acq32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void set_err(Ctl* ctl, uint32_t bits) { atomicOr(&ctl->err, bits); }

// Smallest l with 2^l >= n.
__host__ __device__ __forceinline__ uint32_t ilog2_ceil(uint64_t n) {
  uint32_t l = 0;
  while ((1ull << l) < n) ++l;
  return l;
}

// Adds `flag` (0/1) of every active lane to *ctr with one atomic per wave.
__device__ __forceinline__ void wave_count(uint32_t* ctr, bool flag) {
  const uint64_t bal = __ballot(flag);
  if (bal && (threadIdx.x & 63) == (uint32_t)__builtin_ctzll(__ballot(1))) atomicAdd(ctr, (uint32_t)__popcll(bal));
}

// Stash pool: a bitmap of used entries (bits past the pool size are kept
// set).  The place step takes entries a wave at a time (pool_alloc_wave);
// the rebuild frees them here.
__device__ __forceinline__ void pool_free(uint64_t* used, uint32_t e) {
  atomicAnd((unsigned long long*)&used[e >> 6], ~(1ull << (e & 63)));
}

// The free-address ring of a decomposed store (Sec. 5.2, "Dynamic HBM
// management"): entries are taken at the head (the active lanes of a wave
// that call this together share one atomic) and returned at the tail by
// the batch's finish.  ring_alloc returns kNone when no free entry is left.
__device__ __forceinline__ uint32_t ring_alloc(Ctl* ctl, const uint32_t* ring, uint64_t P) {
  const uint64_t act = __ballot(1);
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t first = (uint32_t)__builtin_ctzll(act);
  uint32_t base = 0;
  if (lane == first) base = atomicAdd(&ctl->ring_take, (uint32_t)__popcll(act));
  base = (uint32_t)__shfl((int)base, (int)first, 64);
  const uint64_t pos = ctl->ring_head + base + __popcll(act & ((1ull << lane) - 1));
  if (pos >= ctl->ring_tail) return kNone;
  return ring[pos % P];
}


__device__ __forceinline__ uint64_t alloc_hash(uint32_t epoch, uint32_t i) {
  uint64_t x = ((uint64_t)epoch << 32) ^ (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
  x ^= x >> 31;
  x *= 0xBF58476D1CE4E5B9ull;
  x ^= x >> 29;
  return x;
}

}  // namespace bolt
