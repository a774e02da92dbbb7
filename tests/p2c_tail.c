/*
 * The bin-load process of the oblivious map under long uniform access, with
 * the two placement rules side by side (TEST INFRASTRUCTURE: a CPU study
 * behind the choice of the default bin capacity; no part of the library).
 *
 * N keys live in B = ceil(N / c) bins.  Every access removes the key from
 * its bin and places it again in the less loaded of a fresh uniform pair of
 * distinct bins, the second bin only when strictly less loaded (Sec. 4.1,
 * Alg. 1's random_remap and P2C_load_balance; Claim 4.2 bounds the largest
 * load by c + O(log log N)).  Accesses come in batches of q uniform keys;
 * repeated keys of a batch move once.  Two rules:
 *
 *   rounds:     the batched rule: all removals of the batch first, then the
 *               moving keys in command order, in rounds of ceil(B/16) keys,
 *               each round choosing on the loads at its start;
 *   sequential: one key at a time, each choosing on the current loads (the
 *               one-at-a-time process the claim analyses).
 *
 * The build fills the bins from empty with the same rule (rounds of
 * ceil(B/16) keys, or one at a time).
 *
 * Output (one JSON line): the largest load ever seen, and for each load L
 * from Z-2 up the number of batch ends whose largest load was at least L.
 *
 * usage: p2c_tail N c q accesses seed rounds|sequential [Z]
 */
#include <inttypes.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static uint64_t rng_state;

/* SplitMix64 (a published 64-bit generator): fast and good enough for a
 * load simulation. */
static uint64_t next_u64(void) {
  uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static uint64_t below(uint64_t n) { return (uint64_t)(((unsigned __int128)next_u64() * n) >> 64); }

/* Load changes that keep the count of bins per load; inc returns the new load. */
static void dec(uint32_t* load, uint64_t* cnt, uint32_t b) {
  cnt[load[b]]--;
  cnt[--load[b]]++;
}

static uint32_t inc(uint32_t* load, uint64_t* cnt, uint32_t b) {
  cnt[load[b]]--;
  if (load[b] >= 254) exit(5);
  cnt[++load[b]]++;
  return load[b];
}

static void fresh_pair(uint64_t B, uint32_t* r1, uint32_t* r2) {
  uint64_t a = below(B);
  *r1 = (uint32_t)a;
  *r2 = (uint32_t)((a + 1 + below(B - 1)) % B);
}

int main(int argc, char** argv) {
  if (argc < 7) {
    fprintf(stderr, "usage: p2c_tail N c q accesses seed rounds|sequential [Z]\n");
    return 2;
  }
  const uint64_t N = strtoull(argv[1], 0, 10), c = strtoull(argv[2], 0, 10), q = strtoull(argv[3], 0, 10);
  const uint64_t accesses = strtoull(argv[4], 0, 10);
  rng_state = strtoull(argv[5], 0, 10);
  const int seq = strcmp(argv[6], "sequential") == 0;
  const uint64_t B = (N + c - 1) / c;
  uint32_t l1 = 0, l2 = 0;
  while ((1ull << l1) < N) ++l1;
  while ((1u << l2) < l1) ++l2;
  const uint32_t Z = argc > 7 ? (uint32_t)atoi(argv[7]) : (uint32_t)(c + l2 + 1);
  const uint64_t rs = seq ? 1 : (B + 15) / 16;

  uint32_t* bin = malloc(N * sizeof(uint32_t));
  uint32_t* load = calloc(B, sizeof(uint32_t));
  uint64_t* stamp = calloc(N, sizeof(uint64_t));
  uint32_t* mv = malloc(q * sizeof(uint32_t));
  uint32_t* ch = malloc((q + 1) * sizeof(uint32_t));
  uint32_t* chb = malloc(((N < rs ? N : rs) + 1) * sizeof(uint32_t));
  uint64_t cnt[256] = {0}; /* bins of each load */
  if (!bin || !load || !stamp || !mv || !ch || !chb) return 3;

  /* build */
  for (uint64_t r0 = 0; r0 < N; r0 += rs) {
    const uint64_t r1 = r0 + rs < N ? r0 + rs : N;
    for (uint64_t i = r0; i < r1; ++i) {
      uint32_t a, b;
      fresh_pair(B, &a, &b);
      chb[i - r0] = load[b] < load[a] ? b : a;
    }
    for (uint64_t i = r0; i < r1; ++i) {
      bin[i] = chb[i - r0];
      load[bin[i]]++;
    }
  }
  uint32_t maxever = 0;
  for (uint64_t b = 0; b < B; ++b) {
    if (load[b] > 255) return 5;
    cnt[load[b]]++;
    maxever = load[b] > maxever ? load[b] : maxever;
  }
  const uint32_t base = Z >= 2 ? Z - 2 : 0;
  uint64_t atleast[8] = {0};
  uint64_t batches = 0;

  for (uint64_t done = 0; done < accesses; done += q) {
    ++batches;
    uint64_t nm = 0;
    for (uint64_t i = 0; i < q; ++i) { /* distinct keys in command order */
      const uint64_t k = below(N);
      if (stamp[k] == batches) continue;
      stamp[k] = batches;
      mv[nm++] = (uint32_t)k;
    }
    if (seq) {
      for (uint64_t i = 0; i < nm; ++i) {
        const uint32_t k = mv[i];
        dec(load, cnt, bin[k]);
        uint32_t a, b;
        fresh_pair(B, &a, &b);
        bin[k] = load[b] < load[a] ? b : a;
        if (inc(load, cnt, bin[k]) > maxever) maxever = load[bin[k]];
      }
    } else {
      for (uint64_t i = 0; i < nm; ++i) dec(load, cnt, bin[mv[i]]);
      for (uint64_t r0 = 0; r0 < nm; r0 += rs) {
        const uint64_t r1 = r0 + rs < nm ? r0 + rs : nm;
        for (uint64_t i = r0; i < r1; ++i) {
          uint32_t a, b;
          fresh_pair(B, &a, &b);
          ch[i - r0] = load[b] < load[a] ? b : a;
        }
        for (uint64_t i = r0; i < r1; ++i) {
          bin[mv[i]] = ch[i - r0];
          if (inc(load, cnt, ch[i - r0]) > maxever) maxever = load[ch[i - r0]];
        }
      }
    }
    uint32_t mx = 255; /* the largest load at the batch end */
    while (mx > 0 && cnt[mx] == 0) --mx;
    for (uint32_t L = base; L < base + 8; ++L)
      if (mx >= L) atleast[L - base]++;
  }
  uint64_t total = 0;
  for (uint64_t b = 0; b < B; ++b) total += load[b];
  if (total != N) {
    fprintf(stderr, "load sum %" PRIu64 " != N\n", total);
    return 4;
  }
  printf("{\"N\": %" PRIu64 ", \"c\": %" PRIu64 ", \"B\": %" PRIu64 ", \"q\": %" PRIu64 ", \"Z\": %u, \"rule\": \"%s\", "
         "\"accesses\": %" PRIu64 ", \"batches\": %" PRIu64 ", \"max_load\": %u, \"batch_ends_at_least\": {",
         N, c, B, q, Z, seq ? "sequential" : "rounds", batches * q, batches, maxever);
  for (uint32_t L = base; L < base + 8; ++L) printf("%s\"%u\": %" PRIu64, L > base ? ", " : "", L, atleast[L - base]);
  printf("}}\n");
  return 0;
}
