/*
 * Stabilizer-tableau oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, byte-per-bit CPU implementation of the phase-space (stabilizer
 * tableau) simulation the paper's Clifford backend is built on (Sec. 2, which
 * cites Aaronson & Gottesman, Phys. Rev. A 70, 052328 (2004), "AG" below).
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
 * use it; the product path never links it.  It shares no code with the GPU
 * library: the two meet only through the seeded circuit arrays.
 *
 * State (AG, "tableau" representation): rows 0..n-1 are destabilizers, rows
 * n..2n-1 stabilizers, row 2n is scratch.  Row i stands for the Pauli product
 * (-1)^r[i] * prod_j P(x[i][j], z[i][j]) with P(0,0)=I, P(1,0)=X, P(0,1)=Z,
 * P(1,1)=Y.  Every entry is one byte holding 0 or 1.
 *
 * Readings where the paper (and its citation) leave a choice open:
 *   - the pivot of a random measurement is the smallest stabilizer row with x=1;
 *   - the random outcome is bit 0 of word 0 of Philox4x64-10 with
 *     key = (seed, 0) and counter = (m, shot, circuit, 0), m = measurement index;
 *   - S is diag(1, i).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int n;
    uint8_t *x;      /* (2n+1) rows x n columns, row-major */
    uint8_t *z;
    uint8_t *r;      /* 2n+1 */
    long anomalies;  /* rowsums whose phase came out odd on a row other than p-n */
} otab;

#define X(t, i, j) ((t)->x[(size_t)(i) * (size_t)(t)->n + (size_t)(j)])
#define Z(t, i, j) ((t)->z[(size_t)(i) * (size_t)(t)->n + (size_t)(j)])

/* ---------------------------------------------------------------- Philox ---
 * Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
 * as 1, 2, 3", SC'11).  One round maps counter (c0,c1,c2,c3) with key (k0,k1)
 * to (hi(B*c2) ^ c1 ^ k0, lo(B*c2), hi(A*c0) ^ c3 ^ k1, lo(A*c0)); the key is
 * bumped by the Weyl constants between rounds.
 */
static void mul128(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo) {
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
    const uint64_t A = 0xD2E7470EE14C6C93ULL, B = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t hA, lA, hB, lB;
        mul128(A, c0, &hA, &lA);
        mul128(B, c2, &hB, &lB);
        uint64_t n0 = hB ^ c1 ^ k0, n1 = lB, n2 = hA ^ c3 ^ k1, n3 = lA;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

int orc_random_bit(uint64_t seed, uint64_t circuit, uint64_t shot, uint64_t m) {
    uint64_t ctr[4] = {m, shot, circuit, 0}, key[2] = {seed, 0}, out[4];
    orc_philox4x64_10(ctr, key, out);
    return (int)(out[0] & 1u);
}

/* -------------------------------------------------------------- tableau --- */
otab *orc_new(int n) {
    otab *t = (otab *)calloc(1, sizeof(otab));
    if (!t) return NULL;
    size_t rows = 2 * (size_t)n + 1;
    t->n = n;
    t->x = (uint8_t *)calloc(rows * (size_t)n, 1);
    t->z = (uint8_t *)calloc(rows * (size_t)n, 1);
    t->r = (uint8_t *)calloc(rows, 1);
    if (!t->x || !t->z || !t->r) { free(t->x); free(t->z); free(t->r); free(t); return NULL; }
    /* |0...0>: destabilizer i = X_i, stabilizer n+i = Z_i, all signs + */
    for (int i = 0; i < n; ++i) {
        X(t, i, i) = 1;
        Z(t, n + i, i) = 1;
    }
    return t;
}

void orc_free(otab *t) {
    if (!t) return;
    free(t->x); free(t->z); free(t->r); free(t);
}

otab *orc_clone(const otab *s) {
    otab *t = orc_new(s->n);
    if (!t) return NULL;
    size_t rows = 2 * (size_t)s->n + 1;
    memcpy(t->x, s->x, rows * (size_t)s->n);
    memcpy(t->z, s->z, rows * (size_t)s->n);
    memcpy(t->r, s->r, rows);
    t->anomalies = s->anomalies;
    return t;
}

int orc_n(const otab *t) { return t->n; }
long orc_anomalies(const otab *t) { return t->anomalies; }

/* Copy out / in the 2n real rows (scratch row excluded). */
void orc_get(const otab *t, uint8_t *x, uint8_t *z, uint8_t *r) {
    size_t cells = 2 * (size_t)t->n * (size_t)t->n;
    memcpy(x, t->x, cells);
    memcpy(z, t->z, cells);
    memcpy(r, t->r, 2 * (size_t)t->n);
}

void orc_set(otab *t, const uint8_t *x, const uint8_t *z, const uint8_t *r) {
    size_t cells = 2 * (size_t)t->n * (size_t)t->n;
    memcpy(t->x, x, cells);
    memcpy(t->z, z, cells);
    memcpy(t->r, r, 2 * (size_t)t->n);
}

/* ---------------------------------------------------------------- gates ---
 * Conjugation rules, one row at a time (AG): the sign picks up x*z for H and
 * S, and x_a z_b (x_b xor z_a xor 1) for CNOT(a -> b).  Each rule reads and
 * writes only its own row, so a whole circuit may be applied row by row.
 *
 * The rest of the Clifford gate set, each from U P U^dagger for the single-
 * qubit Paulis on its qubits:
 *   S^dagger = diag(1, -i): X -> -Y, Y -> X, Z -> Z, so z ^= x and the sign
 *     flips on X (x = 1, z = 0);
 *   X, Y, Z: the Pauli anticommuting with the gate flips sign -- X flips rows
 *     with z = 1, Z rows with x = 1, Y rows with x xor z = 1;
 *   CZ(a, b) = diag(1, 1, 1, -1): X_a -> X_a Z_b, X_b -> Z_a X_b, Z's fixed;
 *     sign flip x_a x_b (z_a xor z_b) (X_a X_b -> Y_a Y_b, Y_a X_b -> -X_a Y_b);
 *   SWAP(a, b): exchanges the two columns, no sign.
 */
static void h_row(otab *t, int i, int a) {
    uint8_t xa = X(t, i, a), za = Z(t, i, a);
    t->r[i] ^= (uint8_t)(xa & za);
    X(t, i, a) = za;
    Z(t, i, a) = xa;
}

static void s_row(otab *t, int i, int a) {
    uint8_t xa = X(t, i, a), za = Z(t, i, a);
    t->r[i] ^= (uint8_t)(xa & za);
    Z(t, i, a) = (uint8_t)(za ^ xa);
}

static void cnot_row(otab *t, int i, int a, int b) {
    uint8_t xa = X(t, i, a), za = Z(t, i, a), xb = X(t, i, b), zb = Z(t, i, b);
    t->r[i] ^= (uint8_t)(xa & zb & (xb ^ za ^ 1));
    X(t, i, b) = (uint8_t)(xb ^ xa);
    Z(t, i, a) = (uint8_t)(za ^ zb);
}

static void sdg_row(otab *t, int i, int a) {
    uint8_t xa = X(t, i, a), za = Z(t, i, a);
    t->r[i] ^= (uint8_t)(xa & (za ^ 1));
    Z(t, i, a) = (uint8_t)(za ^ xa);
}

static void pauli_row(otab *t, int i, int a, int px, int pz) {
    /* sign flips when P(x_a, z_a) anticommutes with P(px, pz) */
    t->r[i] ^= (uint8_t)((X(t, i, a) & pz) ^ (Z(t, i, a) & px));
}

static void cz_row(otab *t, int i, int a, int b) {
    uint8_t xa = X(t, i, a), za = Z(t, i, a), xb = X(t, i, b), zb = Z(t, i, b);
    t->r[i] ^= (uint8_t)(xa & xb & (za ^ zb));
    Z(t, i, a) = (uint8_t)(za ^ xb);
    Z(t, i, b) = (uint8_t)(zb ^ xa);
}

static void swap_row(otab *t, int i, int a, int b) {
    uint8_t xa = X(t, i, a), za = Z(t, i, a);
    X(t, i, a) = X(t, i, b);
    Z(t, i, a) = Z(t, i, b);
    X(t, i, b) = xa;
    Z(t, i, b) = za;
}

void orc_h(otab *t, int a) { for (int i = 0; i < 2 * t->n; ++i) h_row(t, i, a); }
void orc_s(otab *t, int a) { for (int i = 0; i < 2 * t->n; ++i) s_row(t, i, a); }
void orc_cnot(otab *t, int a, int b) { for (int i = 0; i < 2 * t->n; ++i) cnot_row(t, i, a, b); }
void orc_sdg(otab *t, int a) { for (int i = 0; i < 2 * t->n; ++i) sdg_row(t, i, a); }
void orc_x(otab *t, int a) { for (int i = 0; i < 2 * t->n; ++i) pauli_row(t, i, a, 1, 0); }
void orc_y(otab *t, int a) { for (int i = 0; i < 2 * t->n; ++i) pauli_row(t, i, a, 1, 1); }
void orc_z(otab *t, int a) { for (int i = 0; i < 2 * t->n; ++i) pauli_row(t, i, a, 0, 1); }
void orc_cz(otab *t, int a, int b) { for (int i = 0; i < 2 * t->n; ++i) cz_row(t, i, a, b); }
void orc_swap(otab *t, int a, int b) { for (int i = 0; i < 2 * t->n; ++i) swap_row(t, i, a, b); }

/* Layered circuit: per qubit H (if h) then S (if s), then every CNOT pair;
 * applied row by row (each row runs through all layers in order).  Gates on
 * different qubits commute, so within a layer all H's may precede all S's;
 * the per-layer qubit lists are built once, outside the row loop. */
void orc_apply_layers(otab *t, int depth, const uint8_t *h, const uint8_t *s,
                      const uint32_t *ctrl, const uint32_t *tgt, int npairs) {
    int n = t->n;
    int *hl = (int *)malloc(sizeof(int) * ((size_t)depth * n + 1));
    int *sl = (int *)malloc(sizeof(int) * ((size_t)depth * n + 1));
    int *hc = (int *)calloc((size_t)depth + 1, sizeof(int));
    int *sc = (int *)calloc((size_t)depth + 1, sizeof(int));
    if (!hl || !sl || !hc || !sc) { free(hl); free(sl); free(hc); free(sc); return; }
    for (int l = 0; l < depth; ++l)
        for (int q = 0; q < n; ++q) {
            if (h[(size_t)l * n + q]) hl[(size_t)l * n + hc[l]++] = q;
            if (s[(size_t)l * n + q]) sl[(size_t)l * n + sc[l]++] = q;
        }
    for (int i = 0; i < 2 * n; ++i) {
        for (int l = 0; l < depth; ++l) {
            const int *hq = hl + (size_t)l * n, *sq = sl + (size_t)l * n;
            for (int k = 0; k < hc[l]; ++k) h_row(t, i, hq[k]);
            for (int k = 0; k < sc[l]; ++k) s_row(t, i, sq[k]);
            for (int k = 0; k < npairs; ++k)
                cnot_row(t, i, (int)ctrl[(size_t)l * npairs + k], (int)tgt[(size_t)l * npairs + k]);
        }
    }
    free(hl); free(sl); free(hc); free(sc);
}

/* Gate list: op 0 = H(a), 1 = S(a), 2 = CNOT(a -> b), 3 = S^dagger(a),
 * 4 = X(a), 5 = Y(a), 6 = Z(a), 7 = CZ(a, b), 8 = SWAP(a, b).  Returns the
 * index of the first unknown op code (nothing after it applied), or -1. */
long orc_apply_gates(otab *t, long count, const uint8_t *op, const uint32_t *a, const uint32_t *b) {
    for (long k = 0; k < count; ++k) {
        const int qa = (int)a[k], qb = (int)b[k];
        switch (op[k]) {
            case 0: orc_h(t, qa); break;
            case 1: orc_s(t, qa); break;
            case 2: orc_cnot(t, qa, qb); break;
            case 3: orc_sdg(t, qa); break;
            case 4: orc_x(t, qa); break;
            case 5: orc_y(t, qa); break;
            case 6: orc_z(t, qa); break;
            case 7: orc_cz(t, qa, qb); break;
            case 8: orc_swap(t, qa, qb); break;
            default: return k;
        }
    }
    return -1;
}

/* ---------------------------------------------------------- g / rowsum ---
 * g(x1,z1,x2,z2): exponent to which i is raised when the single-qubit Paulis
 * P(x1,z1) and P(x2,z2) are multiplied (AG).
 */
int orc_g(int x1, int z1, int x2, int z2) {
    if (x1 == 0 && z1 == 0) return 0;
    if (x1 == 1 && z1 == 1) return z2 - x2;
    if (x1 == 1 && z1 == 0) return z2 * (2 * x2 - 1);
    return x2 * (1 - 2 * z2); /* x1 == 0, z1 == 1 */
}

/* rowsum(h, i): row h <- row i * row h with the sign tracked mod 4 (AG). */
static void rowsum_raw(otab *t, int h, int i, int *e_out) {
    int n = t->n;
    long e = 2L * t->r[h] + 2L * t->r[i];
    for (int j = 0; j < n; ++j)
        e += orc_g(X(t, i, j), Z(t, i, j), X(t, h, j), Z(t, h, j));
    e %= 4;
    if (e < 0) e += 4;
    *e_out = (int)e;
    t->r[h] = (uint8_t)(e == 2 ? 1 : 0);
    for (int j = 0; j < n; ++j) {
        X(t, h, j) ^= X(t, i, j);
        Z(t, h, j) ^= Z(t, i, j);
    }
}

/* Exported single rowsum; returns e mod 4 (0 or 2 when the rows commute). */
int orc_rowsum(otab *t, int h, int i) {
    int e;
    rowsum_raw(t, h, i, &e);
    return e;
}

/* ----------------------------------------------------------- measurement ---
 * Measurement of the single-qubit Pauli P_a = P(px, pz) on qubit a (AG's
 * Z-measurement, px = 0 and pz = 1, with "row i anticommutes with Z_a", x_ia =
 * 1, read as "row i anticommutes with P_a": x_ia pz xor z_ia px = 1; the
 * argument of AG carries over unchanged to any Pauli).  Returns the outcome
 * bit (0 for eigenvalue +1); *kind is set to 1 when the outcome was random, 0
 * when it was determined by the state.
 */
static int anticommutes(const otab *t, int i, int a, int px, int pz) {
    return (X(t, i, a) & pz) ^ (Z(t, i, a) & px);
}

int orc_measure_pauli(otab *t, int a, int px, int pz, uint64_t seed, uint64_t circuit,
                      uint64_t shot, uint64_t m, int *kind) {
    int n = t->n;
    int p = -1;
    for (int i = n; i < 2 * n; ++i)
        if (anticommutes(t, i, a, px, pz)) { p = i; break; }

    if (p >= 0) {
        /* random: multiply the pivot into every other row that anticommutes
           with P_a, move the pivot into its destabilizer slot, and replace it
           by +-P_a with a fresh random sign */
        for (int i = 0; i < 2 * n; ++i) {
            if (i == p || !anticommutes(t, i, a, px, pz)) continue;
            int e;
            rowsum_raw(t, i, p, &e);
            if ((e & 1) && i != p - n) t->anomalies++;
        }
        memcpy(&X(t, p - n, 0), &X(t, p, 0), (size_t)n);
        memcpy(&Z(t, p - n, 0), &Z(t, p, 0), (size_t)n);
        t->r[p - n] = t->r[p];
        memset(&X(t, p, 0), 0, (size_t)n);
        memset(&Z(t, p, 0), 0, (size_t)n);
        X(t, p, a) = (uint8_t)px;
        Z(t, p, a) = (uint8_t)pz;
        t->r[p] = (uint8_t)orc_random_bit(seed, circuit, shot, m);
        if (kind) *kind = 1;
        return t->r[p];
    }

    /* deterministic: accumulate the product of the stabilizers whose
       destabilizer partner anticommutes with P_a in the scratch row */
    int sc = 2 * n;
    memset(&X(t, sc, 0), 0, (size_t)n);
    memset(&Z(t, sc, 0), 0, (size_t)n);
    t->r[sc] = 0;
    for (int i = 0; i < n; ++i) {
        if (!anticommutes(t, i, a, px, pz)) continue;
        int e;
        rowsum_raw(t, sc, i + n, &e);
        if (e & 1) t->anomalies++;
    }
    if (kind) *kind = 0;
    return t->r[sc];
}

/* Z-measurement of qubit a (AG). */
int orc_measure(otab *t, int a, uint64_t seed, uint64_t circuit, uint64_t shot,
                uint64_t m, int *kind) {
    return orc_measure_pauli(t, a, 0, 1, seed, circuit, shot, m, kind);
}

/* Reset of qubit a to |0>: Z-measure it, and where the outcome is 1 apply X
 * (which maps the post-measurement eigenstate -Z_a to +Z_a).  Returns the
 * measured outcome. */
int orc_reset(otab *t, int a, uint64_t seed, uint64_t circuit, uint64_t shot, uint64_t m,
              int *kind) {
    int out = orc_measure(t, a, seed, circuit, shot, m, kind);
    if (out) orc_x(t, a);
    return out;
}

/*
 * Whole circuit for one shot: gates on a fresh |0...0>, then measure
 * qubits[0..k) in order with measurement index m = position.  Outcomes and
 * kinds are written to out[k] / kind[k]; if x, z, r are non-NULL the final
 * tableau (2n rows) is copied out.  Returns 0, or -1 on allocation failure.
 */
int orc_run_shot(int n, int depth, const uint8_t *h, const uint8_t *s,
                 const uint32_t *ctrl, const uint32_t *tgt, int npairs,
                 int k, const uint32_t *qubits, uint64_t seed, uint64_t circuit,
                 uint64_t shot, uint8_t *out, uint8_t *kind,
                 uint8_t *x, uint8_t *z, uint8_t *r) {
    otab *t = orc_new(n);
    if (!t) return -1;
    orc_apply_layers(t, depth, h, s, ctrl, tgt, npairs);
    for (int m = 0; m < k; ++m) {
        int kd;
        out[m] = (uint8_t)orc_measure(t, (int)qubits[m], seed, circuit, shot, (uint64_t)m, &kd);
        if (kind) kind[m] = (uint8_t)kd;
    }
    if (x && z && r) orc_get(t, x, z, r);
    orc_free(t);
    return 0;
}

/* Measure qubits[0..k) on the given tableau (in place), indices m0.. */
void orc_measure_list(otab *t, int k, const uint32_t *qubits, uint64_t seed,
                      uint64_t circuit, uint64_t shot, uint64_t m0,
                      uint8_t *out, uint8_t *kind) {
    for (int m = 0; m < k; ++m) {
        int kd;
        out[m] = (uint8_t)orc_measure(t, (int)qubits[m], seed, circuit, shot, m0 + (uint64_t)m, &kd);
        if (kind) kind[m] = (uint8_t)kd;
    }
}
