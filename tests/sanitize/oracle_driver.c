/* Host sanitizer run of the oracle (test infrastructure): built together
 * with oracle/chp.c under -fsanitize=address,undefined and run on random
 * circuits of several sizes, with gates of the whole set, measurements in all
 * three bases (random and deterministic branches), resets, clones, get/set
 * round trips and whole shots.  Any out-of-bounds access, use after free,
 * leak or undefined behaviour aborts the run with a report. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct otab otab;
otab *orc_new(int n);
void orc_free(otab *t);
otab *orc_clone(const otab *s);
long orc_anomalies(const otab *t);
void orc_get(const otab *t, uint8_t *x, uint8_t *z, uint8_t *r);
void orc_set(otab *t, const uint8_t *x, const uint8_t *z, const uint8_t *r);
long orc_apply_gates(otab *t, long count, const uint8_t *op, const uint32_t *a, const uint32_t *b);
void orc_apply_layers(otab *t, int depth, const uint8_t *h, const uint8_t *s, const uint32_t *ctrl,
                      const uint32_t *tgt, int npairs);
int orc_measure_pauli(otab *t, int a, int px, int pz, uint64_t seed, uint64_t circuit, uint64_t shot,
                      uint64_t m, int *random);
int orc_reset(otab *t, int a, uint64_t seed, uint64_t circuit, uint64_t shot, uint64_t m, int *random);
int orc_run_shot(int n, int depth, const uint8_t *h, const uint8_t *s, const uint32_t *ctrl,
                 const uint32_t *tgt, int npairs, int k, const uint32_t *qubits, uint64_t seed,
                 uint64_t circuit, uint64_t shot, uint8_t *out, uint8_t *kind, uint8_t *x, uint8_t *z,
                 uint8_t *r);

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint32_t rnd(uint32_t m) {   /* xorshift64*, modulo m */
  rng_state ^= rng_state >> 12;
  rng_state ^= rng_state << 25;
  rng_state ^= rng_state >> 27;
  return (uint32_t)((rng_state * 0x2545F4914F6CDD1Dull) >> 33) % m;
}

static int one_size(int n) {
  otab *t = orc_new(n);
  if (!t) return 1;
  const long count = 12L * n + 20;
  uint8_t *op = malloc(count);
  uint32_t *a = malloc(count * 4), *b = malloc(count * 4);
  for (long i = 0; i < count; ++i) {
    op[i] = (uint8_t)rnd(n > 1 ? 9 : 7);
    if (n == 1 && (op[i] == 2)) op[i] = 0;
    a[i] = rnd(n);
    b[i] = n > 1 ? (a[i] + 1 + rnd(n - 1)) % n : 0;
  }
  if (orc_apply_gates(t, count, op, a, b) != -1) return 1;   /* -1: every op applied */
  for (int m = 0; m < 2 * n; ++m) {
    int random = 0;
    const int basis = (int)rnd(3);
    orc_measure_pauli(t, (int)rnd(n), basis != 2, basis != 0, 7, 1, 0, (uint64_t)m, &random);
    if (m % 5 == 4) orc_reset(t, (int)rnd(n), 7, 1, 0, (uint64_t)m, &random);
  }
  otab *c = orc_clone(t);
  uint8_t *x = malloc((size_t)2 * n * n), *z = malloc((size_t)2 * n * n), *r = malloc(2 * n);
  orc_get(c, x, z, r);
  orc_set(t, x, z, r);
  const int depth = 5, np = n / 2;
  uint8_t *h = malloc((size_t)depth * n), *s = malloc((size_t)depth * n);
  uint32_t *ct = malloc((size_t)depth * (np + 1) * 4), *tg = malloc((size_t)depth * (np + 1) * 4);
  uint32_t *perm = malloc((size_t)n * 4);
  for (int l = 0; l < depth; ++l) {
    for (int q = 0; q < n; ++q) {
      h[l * n + q] = (uint8_t)rnd(2);
      s[l * n + q] = (uint8_t)rnd(2);
      perm[q] = (uint32_t)q;
    }
    for (int q = n - 1; q > 0; --q) {
      const int j = (int)rnd((uint32_t)q + 1);
      const uint32_t v = perm[q]; perm[q] = perm[j]; perm[j] = v;
    }
    for (int k = 0; k < np; ++k) {
      ct[l * np + k] = perm[2 * k];
      tg[l * np + k] = perm[2 * k + 1];
    }
  }
  orc_apply_layers(t, depth, h, s, ct, tg, np);
  uint32_t *qs = malloc((size_t)n * 4);
  for (int q = 0; q < n; ++q) qs[q] = (uint32_t)q;
  uint8_t *out = malloc(n), *kind = malloc(n);
  if (orc_run_shot(n, depth, h, s, ct, tg, np, n, qs, 9, 2, 3, out, kind, x, z, r) != 0) return 1;
  const long anomalies = orc_anomalies(t) + orc_anomalies(c);
  orc_free(c);
  orc_free(t);
  free(op); free(a); free(b); free(x); free(z); free(r); free(h); free(s); free(ct); free(tg);
  free(perm); free(qs); free(out); free(kind);
  return anomalies != 0;
}

int main(void) {
  const int sizes[] = {1, 2, 3, 5, 31, 32, 33, 63, 64, 65, 100, 129};
  for (size_t i = 0; i < sizeof(sizes) / sizeof(sizes[0]); ++i)
    if (one_size(sizes[i])) {
      fprintf(stderr, "oracle run failed at n = %d\n", sizes[i]);
      return 1;
    }
  printf("oracle sanitizer run ok\n");
  return 0;
}
