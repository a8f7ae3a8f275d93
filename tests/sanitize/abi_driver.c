/* Host sanitizer run of the library's host code (test infrastructure): the
 * gate encoders, argument checks, size queries and error paths of the C ABI,
 * built with -fsanitize=address,undefined on the host side only and run on a
 * machine with or without a GPU (nothing here launches a kernel).  Any
 * out-of-bounds access, leak or undefined behaviour aborts with a report;
 * a wrong return code exits non-zero with a message. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "cliff.h"

static int failures = 0;
#define EXPECT(cond)                                                              \
  do {                                                                            \
    if (!(cond)) {                                                                \
      fprintf(stderr, "%s:%d: expected %s (%s)\n", __FILE__, __LINE__, #cond,     \
              cliff_last_error());                                                \
      ++failures;                                                                 \
    }                                                                             \
  } while (0)

static uint64_t st = 0x243F6A8885A308D3ull;
static uint32_t rnd(uint32_t m) {
  st ^= st >> 12;
  st ^= st << 25;
  st ^= st >> 27;
  return (uint32_t)((st * 0x2545F4914F6CDD1Dull) >> 33) % m;
}

static void layers(uint32_t n, uint32_t depth) {
  const uint32_t np = n / 2;
  uint8_t *h = malloc((size_t)depth * n + 1), *s = malloc((size_t)depth * n + 1);
  uint32_t *c = malloc((size_t)depth * np * 4 + 4), *t = malloc((size_t)depth * np * 4 + 4);
  uint32_t *perm = malloc((size_t)n * 4);
  for (uint32_t l = 0; l < depth; ++l) {
    for (uint32_t q = 0; q < n; ++q) {
      h[l * n + q] = (uint8_t)rnd(2);
      s[l * n + q] = (uint8_t)rnd(2);
      perm[q] = q;
    }
    for (uint32_t q = n - 1; q > 0; --q) {
      const uint32_t j = rnd(q + 1), v = perm[q];
      perm[q] = perm[j];
      perm[j] = v;
    }
    for (uint32_t k = 0; k < np; ++k) {
      c[l * np + k] = perm[2 * k];
      t[l * np + k] = perm[2 * k + 1];
    }
  }
  size_t nops = 0;
  uint32_t *offs = malloc((size_t)(depth + 1) * 4);
  EXPECT(cliff_encode_layers(n, h, s, c, t, np, depth, NULL, 0, offs, &nops) == CLIFF_OK);
  uint64_t *ops = malloc(nops * 8 + 8);
  size_t got = 0;
  EXPECT(cliff_encode_layers(n, h, s, c, t, np, depth, ops, nops, offs, &got) == CLIFF_OK);
  EXPECT(got == nops);
  if (nops > 0) EXPECT(cliff_encode_layers(n, h, s, c, t, np, depth, ops, nops - 1, offs, &got) != CLIFF_OK);
  if (np > 0) {   /* a qubit twice in one layer, then a qubit out of range */
    const uint32_t keep = t[0];
    t[0] = c[0];
    EXPECT(cliff_encode_layers(n, h, s, c, t, np, depth, ops, nops, offs, &got) == CLIFF_EINVAL);
    t[0] = n;
    EXPECT(cliff_encode_layers(n, h, s, c, t, np, depth, ops, nops, offs, &got) == CLIFF_EINVAL);
    t[0] = keep;
  }
  free(h); free(s); free(c); free(t); free(perm); free(offs); free(ops);
}

static void gate_lists(uint32_t n, size_t count) {
  uint8_t *op = malloc(count + 1);
  uint32_t *a = malloc(count * 4 + 4), *b = malloc(count * 4 + 4);
  for (size_t i = 0; i < count; ++i) {
    op[i] = (uint8_t)rnd(n > 1 ? 9 : 7);
    if (n == 1 && op[i] == CLIFF_OP_CNOT) op[i] = CLIFF_OP_H;
    a[i] = rnd(n);
    b[i] = n > 1 ? (a[i] + 1 + rnd(n - 1)) % n : 0;
  }
  size_t nops = 0;
  uint32_t depth = 0;
  EXPECT(cliff_encode_gates(n, op, a, b, count, NULL, 0, NULL, 0, &nops, &depth) == CLIFF_OK);
  uint64_t *ops = malloc(nops * 8 + 8);
  uint32_t *offs = malloc((size_t)(depth + 1) * 4);
  size_t n2 = 0;
  uint32_t d2 = 0;
  EXPECT(cliff_encode_gates(n, op, a, b, count, ops, nops, offs, depth + 1, &n2, &d2) == CLIFF_OK);
  EXPECT(n2 == nops && d2 == depth);
  if (depth > 0)
    EXPECT(cliff_encode_gates(n, op, a, b, count, ops, nops, offs, depth, &n2, &d2) == CLIFF_ENOMEM);
  if (count > 0) {
    const uint8_t keep = op[0];
    op[0] = 9;   /* unknown op */
    EXPECT(cliff_encode_gates(n, op, a, b, count, ops, nops, offs, depth + 1, &n2, &d2) == CLIFF_EINVAL);
    op[0] = CLIFF_OP_CZ;   /* a two-qubit gate on one qubit */
    const uint32_t kb = b[0];
    b[0] = a[0];
    EXPECT(cliff_encode_gates(n, op, a, b, count, ops, nops, offs, depth + 1, &n2, &d2) == CLIFF_EINVAL);
    b[0] = kb;
    op[0] = keep;
  }
  free(op); free(a); free(b); free(ops); free(offs);
}

int main(void) {
  const uint32_t sizes[] = {1, 2, 3, 31, 32, 33, 64, 65, 130, 1000};
  for (size_t i = 0; i < sizeof(sizes) / sizeof(sizes[0]); ++i) {
    layers(sizes[i], 7);
    gate_lists(sizes[i], 40 * sizes[i] + 3);
  }
  /* size queries and argument checks that need no device */
  EXPECT(cliff_tab_bytes(10000, 1) > 2 * 10000ull * 320 * 8);
  EXPECT(cliff_tab_bytes(1, 1024) > 0);
  EXPECT(cliff_batch_work_bytes() > 0);
  EXPECT(cliff_tab_bind(NULL, 8, 1, NULL, 0, NULL) == CLIFF_EINVAL);
  EXPECT(cliff_apply_gates(NULL, NULL, NULL, NULL, 0) == CLIFF_EINVAL);
  EXPECT(cliff_measure(NULL, NULL, 0, 0, 0, 0, 0, NULL, NULL) == CLIFF_EINVAL);
  EXPECT(cliff_encode_layers(0, NULL, NULL, NULL, NULL, 0, 0, NULL, 0, NULL, NULL) == CLIFF_EINVAL);
  for (int code = 0; code >= -6; --code) EXPECT(cliff_strerror(code) != NULL);
  EXPECT(cliff_last_error() != NULL);
  if (failures) {
    fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  printf("abi sanitizer run ok\n");
  return 0;
}
