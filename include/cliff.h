/*
 * cliff.h -- C ABI of the MI355X (gfx950) stabilizer-tableau library.
 *
 * The library simulates Clifford circuits in the phase-space (stabilizer
 * tableau) formalism that the paper's Clifford backend is built on (Sec. 2,
 * "Simulation of Clifford circuits", which cites Aaronson & Gottesman,
 * Phys. Rev. A 70, 052328 (2004) for the method).  A tableau on n qubits has
 * 2n rows: rows 0..n-1 are destabilizers, rows n..2n-1 stabilizers; row i is
 * the signed Pauli product (-1)^r_i * prod_j P(x_ij, z_ij).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Return value: 0 (CLIFF_OK) or a negative CLIFF_E* code.  No call aborts
 *    or throws across this boundary; cliff_last_error() gives a message for the
 *    most recent failure on the calling thread.
 *  - Device memory belongs to the caller.  A tableau is a view bound onto one
 *    caller-owned device buffer of cliff_tab_bytes(n, shots) bytes; the library
 *    never frees it.  The context owns only its own staging buffers and the
 *    register-resident measurement's chunk scratch (allocated at the first
 *    such measurement, grown to the largest tableau shape the context has
 *    measured: about 270 MB at n = 4,096, 2.2 GB at n = 10,000; freed by
 *    cliff_ctx_destroy).
 *  - Host pointers are read (inputs) or written (outputs) before the call
 *    returns.  Calls that return host data synchronize the context stream;
 *    the others only enqueue work on it.
 *  - Qubit indices are 0-based.  Row bits are packed LSB-first into 64-bit
 *    words per qubit column (word w of column j holds rows 64w..64w+63).
 *  - Shots: a tableau carries `shots` independent sign columns.  X/Z bits
 *    never depend on signs or outcomes, so all shots share one X/Z sweep and
 *    only the signs (and outcomes) differ per shot.
 *  - Random outcomes: bit 0 of word 0 of Philox4x64-10 with key (seed, 0) and
 *    counter (m, shot, circuit, 0), m = measurement index.
 */
#ifndef CLIFF_H
#define CLIFF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CLIFF_OK 0
#define CLIFF_EINVAL (-1)   /* bad argument: qubit >= n, two-qubit gate a == b, bad op, NULL, size */
#define CLIFF_ENOMEM (-2)   /* buffer too small / host allocation failed / budget exceeded */
#define CLIFF_EDEVICE (-3)  /* HIP runtime error (message in cliff_last_error) */
#define CLIFF_EBUSY (-4)    /* resource in use (e.g. admission slots full) */
#define CLIFF_EINTERNAL (-5) /* a device-side consistency check failed */

/* Gate op codes of cliff_apply_gates. */
#define CLIFF_OP_H 0
#define CLIFF_OP_S 1
#define CLIFF_OP_CNOT 2
#define CLIFF_OP_SDG 3    /* S^dagger = diag(1, -i) */
#define CLIFF_OP_X 4
#define CLIFF_OP_Y 5
#define CLIFF_OP_Z 6
#define CLIFF_OP_CZ 7
#define CLIFF_OP_SWAP 8

/* Measurement bases of cliff_measure_bases. */
#define CLIFF_BASIS_Z 0
#define CLIFF_BASIS_X 1
#define CLIFF_BASIS_Y 2

typedef struct cliff_ctx cliff_ctx;
typedef struct cliff_tab cliff_tab;

/* Message for the last failing call on this thread (static storage). */
const char *cliff_last_error(void);
/* Name of a CLIFF_E* code. */
const char *cliff_strerror(int code);

/* Context: one device and one HIP stream (borrowed; may be NULL for the
 * default stream).  All work of tableaux bound to it is ordered on that
 * stream: a call's kernels may also run on a second stream the context owns
 * (the register-resident measurement overlaps a chunk's finalize with the
 * next chunk), but the bound stream waits for them before the call's later
 * work, so everything enqueued afterwards on the bound stream sees the
 * results.  Owns small staging buffers, that stream and its events (created
 * here) and the measurement chunk scratch (see above).  Destroy synchronizes
 * both streams before it releases them. */
int cliff_ctx_create(int device, void *hip_stream, cliff_ctx **out);
int cliff_ctx_destroy(cliff_ctx *ctx);
/* Block until all work enqueued by the context has finished. */
int cliff_sync(cliff_ctx *ctx);
/* Number of compute units of the context's device. */
int cliff_ctx_num_cus(const cliff_ctx *ctx);

/* Roofline calibration (a measurement aid, not part of the simulation):
 * runs a kernel on every CU of the context's device, on its stream, and writes
 * the rate it reached to *out.  CLIFF_CAL_LDS: bytes per second of
 * conflict-free 16-byte LDS reads; CLIFF_CAL_VALU: 32-bit bitwise VALU lane
 * operations per second (v_xor_b32, independent chains).  Allocates and frees
 * 4 KB of device memory; synchronizes.  CLIFF_EINVAL for another kind. */
#define CLIFF_CAL_LDS 0
#define CLIFF_CAL_VALU 1
int cliff_calibrate(cliff_ctx *ctx, int kind, double *out);

/* Gate-stream strategy.  AUTO: one launch for all layers when 8n bytes (32
 * rows of every column) fit in LDS, else one launch per layer.  PER_LAYER:
 * always one launch per layer.  FUSED: always one launch (EINVAL if n is too
 * large).  Results are identical; only speed differs. */
#define CLIFF_GATES_AUTO 0
#define CLIFF_GATES_PER_LAYER 1
#define CLIFF_GATES_FUSED 2
int cliff_ctx_set_gate_mode(cliff_ctx *ctx, int mode);

/* Measurement strategy.  PERSISTENT: the register-resident path (the tableau
 * held in registers and LDS of up to 256 compute units for a chunk of
 * measurements, one rowsum sweep per measurement); EINVAL when the tableau
 * shape does not fit (ceil(2n/64) <= 320, i.e. n <= 10240).  BLOCKED: the
 * register-resident path where each chunk's leading run of random
 * measurements is applied in blocks of up to 32 as one low-rank update (the
 * per-measurement kernels take the chunk's remaining measurements from its
 * first deterministic one); where the blocked launch shape does not fit
 * (n in (2040 L, 2048 L] for L = ceil(2n/4096), e.g. n = 2041..2048,
 * 8161..8192, 10201..10240) it is PERSISTENT.  STEP: one kernel per
 * measurement.  AUTO: BLOCKED for n >= 2048, PERSISTENT below, STEP where
 * neither fits.  Results are identical; only speed differs.  A measure-all of
 * a dense state at n = 10,000 takes 16.1 ms with BLOCKED against 38.7 ms with
 * PERSISTENT (6,000: 9.5 against 16.5 ms; 2,100: 4.0 against 4.6 ms); a GHZ
 * measure-all (n - 1 of n outcomes deterministic) takes 61 ms with the
 * register-resident path at n = 10,000 against 125 ms with STEP.  From
 * n = 3,000 the blocked pass works in chunks of 2048 measurements, whose
 * scratch (about 5.6 GB at n = 10,000) the context allocates at its first
 * such call; if device memory refuses it, the call runs with the
 * per-measurement path's smaller chunks instead (same results;
 * cliff_last_error then names the refused allocation). */
#define CLIFF_MEASURE_AUTO 0
#define CLIFF_MEASURE_STEP 1
#define CLIFF_MEASURE_PERSISTENT 2
#define CLIFF_MEASURE_BLOCKED 3
int cliff_ctx_set_measure_mode(cliff_ctx *ctx, int mode);

/* Failure handling of the register-resident path.  Its workgroups wait for
 * each other's published columns with bounded waits; a wait that runs out
 * raises a device-side abort flag, every workgroup leaves, later chunks of the
 * pass skip their work, and the tableau's contents are undefined (initialize
 * or import it again).  The flag stays raised until a synchronizing call
 * reports CLIFF_EINTERNAL: cliff_measure, cliff_tab_read_outcomes,
 * cliff_sample, cliff_tab_anomalies or cliff_tab_counters; that report
 * lowers it.
 * cliff_ctx_inject_abort (a test aid for this path): counting the
 * measurements the context performs from now on from 0 (in any tableau, by
 * any measuring call), every workgroup gives up at measurement `at` exactly as
 * if a wait had run out, provided that measurement runs on the
 * register-resident path; then the setting is spent.  UINT64_MAX (the
 * default) injects nothing. */
int cliff_ctx_inject_abort(cliff_ctx *ctx, uint64_t at);

/* Bytes of device memory a tableau of n qubits with `shots` sign columns needs:
 * X, Z, signs, the per-measurement path's scratch and the outcome staging
 * (the register-resident path's chunk scratch belongs to the context). */
size_t cliff_tab_bytes(uint32_t n, uint32_t shots);

/* Bind a tableau view onto caller-owned device memory `dev` of `bytes` bytes
 * (>= cliff_tab_bytes(n, shots), 256-byte aligned).  Does not allocate device
 * memory and does not initialise it (call cliff_tab_init_zero or _import). */
int cliff_tab_bind(cliff_ctx *ctx, uint32_t n, uint32_t shots, void *dev, size_t bytes,
                   cliff_tab **out);
int cliff_tab_unbind(cliff_tab *tab);
int cliff_tab_info(const cliff_tab *tab, uint32_t *n, uint32_t *shots);

/* |0...0>: destabilizer i = X_i, stabilizer n+i = Z_i, all signs + (the
 * initial tableau of the phase-space method, Sec. 2 / AG). */
int cliff_tab_init_zero(cliff_tab *tab);

/* Apply gates in order.  op[k] is a CLIFF_OP_* code; a[k] is the qubit (the
 * CNOT control), b[k] the second qubit of CNOT (target), CZ and SWAP (ignored
 * otherwise).  Update rules per row (AG, via Sec. 2; the others from
 * conjugating each single-qubit Pauli by the gate):
 *   H(a): r ^= x_a z_a, swap x_a and z_a;   S(a): r ^= x_a z_a, z_a ^= x_a;
 *   CNOT(a->b): r ^= x_a z_b (x_b ^ z_a ^ 1), x_b ^= x_a, z_a ^= z_b;
 *   SDG(a): r ^= x_a (z_a ^ 1), z_a ^= x_a;
 *   X(a): r ^= z_a;   Y(a): r ^= x_a ^ z_a;   Z(a): r ^= x_a;
 *   CZ(a,b): r ^= x_a x_b (z_a ^ z_b), z_a ^= x_b, z_b ^= x_a;
 *   SWAP(a,b): exchange columns a and b.
 * Runs of single-qubit gates on a qubit are composed into one column update
 * on the host.  Validated on the host before any launch (EINVAL on bad op /
 * qubit / a == b for a two-qubit gate). */
int cliff_apply_gates(cliff_tab *tab, const uint8_t *op, const uint32_t *a, const uint32_t *b,
                      size_t count);

/* Apply `depth` layers.  Layer l: for every qubit q, H if h[l*n+q], then S if
 * s[l*n+q]; then CNOT(ctrl[l*npairs+k] -> tgt[l*npairs+k]) for k < npairs.
 * The qubits of one layer's pairs must be distinct (EINVAL otherwise). */
int cliff_apply_layers(cliff_tab *tab, const uint8_t *h, const uint8_t *s, const uint32_t *ctrl,
                       const uint32_t *tgt, uint32_t npairs, uint32_t depth);

/* Pre-encoded gate stream for repeated or device-resident use.
 * cliff_encode_layers writes the library's op words for the layers above into
 * ops (capacity in 64-bit words) and layer boundaries into offs[depth+1];
 * *nops receives the word count.  With ops == NULL it only reports *nops.
 * cliff_apply_encoded runs such a stream from DEVICE memory dev_ops, with the
 * host array offs[depth+1] of layer boundaries. */
int cliff_encode_layers(uint32_t n, const uint8_t *h, const uint8_t *s, const uint32_t *ctrl,
                        const uint32_t *tgt, uint32_t npairs, uint32_t depth, uint64_t *ops,
                        size_t cap, uint32_t *offs, size_t *nops);
int cliff_apply_encoded(cliff_tab *tab, const uint64_t *dev_ops, const uint32_t *offs,
                        uint32_t depth);

/* Encode a gate list (op codes and rules of cliff_apply_gates) into the
 * library's op words and layer boundaries, for device-resident reuse with
 * cliff_apply_encoded / cliff_apply_encoded_many.  *nops and *depth receive
 * the sizes; ops (capacity ops_cap words) and offs (offs_cap entries, depth
 * + 1 needed) may be NULL to query them only.  EINVAL as cliff_apply_gates;
 * ENOMEM if a non-NULL output is too small (sizes still reported). */
int cliff_encode_gates(uint32_t n, const uint8_t *op, const uint32_t *a, const uint32_t *b,
                       size_t count, uint64_t *ops, size_t ops_cap, uint32_t *offs, size_t offs_cap,
                       size_t *nops, uint32_t *depth);

/* Gates only, on many tableaux in one launch (the paper's Fig. 2a workload:
 * many random Clifford circuits, no measurement).  Every tableau is split
 * into groups of rows_per_group rows (32, 64 or 128; 0 picks one from the
 * sizes); one workgroup holds its group of every column in LDS and runs all
 * layers.  tabs[0..count): distinct tableaux bound to one context,
 * 2 n rows_per_group/8 bytes <= 159 KiB (n <= 20,352 at 32 rows, 10,176 at
 * 64, 5,088 at 128), count <= 65,535.
 * _encoded_many: tableau i runs the encoded stream at DEVICE pointer
 * dev_ops[i] (caller-owned, unchanged until the launch has run) with the HOST
 * array offs[i][0..depths[i]] of layer boundaries.  _gates_many: tableau i
 * runs the gate list (op[i], a[i], b[i], counts[i]) as cliff_apply_gates
 * would, encoded on the host.  Only enqueues work (the staged descriptors
 * and offsets are copied before the call returns).  EINVAL on a NULL array
 * or tableau, a repeated tableau, tableaux on different contexts, a size
 * that does not fit, bad ops, or decreasing offsets. */
int cliff_apply_encoded_many(cliff_tab *const *tabs, const uint64_t *const *dev_ops,
                             const uint32_t *const *offs, const uint32_t *depths, size_t count,
                             int rows_per_group);
int cliff_apply_gates_many(cliff_tab *const *tabs, const uint8_t *const *op, const uint32_t *const *a,
                           const uint32_t *const *b, const size_t *counts, size_t count,
                           int rows_per_group);

/* Z-measure qubits[0..k) in order (AG measurement, via Sec. 2).  Measurement
 * i has index m = m0 + i for the random-bit counter.  Random branch: the pivot
 * is the smallest stabilizer row with x_a = 1; every other row with x_a = 1
 * is multiplied by it (rowsum, phase function g, mod 4); the pivot moves to
 * its destabilizer slot and becomes +-Z_a with the Philox bit as sign and
 * outcome.  Deterministic branch: the outcome is the sign of the product of
 * the stabilizers whose destabilizer has x_a = 1; the tableau is unchanged.
 * All `shots` sign columns are measured at once: shot s uses counter shot
 * index shot0 + s.  host_out (nullable) receives outcomes as uint8 [shots][k];
 * host_random (nullable) receives 1 where measurement i was random. */
int cliff_measure(cliff_tab *tab, const uint32_t *qubits, size_t k, uint64_t seed,
                  uint64_t circuit, uint64_t shot0, uint64_t m0, uint8_t *host_out,
                  uint8_t *host_random);

/* Measure the single-qubit Pauli bases[i] (CLIFF_BASIS_Z, _X or _Y) on
 * qubits[i], in order, with the conventions of cliff_measure (outcome 0 =
 * eigenvalue +1, random branch: the measured Pauli with the Philox bit as
 * sign).  Measuring P_a is measuring Z_a after a Clifford U with U P_a U^dag =
 * Z_a (X: H; Y: S^dagger then H) and undoing U afterwards; the library does
 * exactly that, per run of distinct qubits: one gate layer, a Z-measurement
 * pass, and the inverse layer.  EINVAL on a bad basis or qubit. */
int cliff_measure_bases(cliff_tab *tab, const uint32_t *qubits, const uint8_t *bases, size_t k,
                        uint64_t seed, uint64_t circuit, uint64_t shot0, uint64_t m0,
                        uint8_t *host_out, uint8_t *host_random);

/* Mid-circuit measurement into a DEVICE record (caller-owned, at least
 * shots * ld bytes): as cliff_measure, but the outcome of measurement i of
 * shot s is written to dev_record[s * ld + col0 + i] (0/1) and, if
 * dev_random is not NULL, the random flag to dev_random[col0 + i] (device).
 * Only enqueues work; nothing is copied to the host.  EINVAL if
 * col0 + k > ld or on a bad qubit. */
int cliff_measure_record(cliff_tab *tab, const uint32_t *qubits, size_t k, uint64_t seed,
                         uint64_t circuit, uint64_t shot0, uint64_t m0, uint8_t *dev_record,
                         size_t ld, size_t col0, uint8_t *dev_random);

/* Reset qubits[0..k) to |0>: Z-measure each (recorded exactly as
 * cliff_measure_record, measurement index m0 + i) and apply X in every shot
 * whose outcome was 1.  X flips only signs, so all shots keep one set of X/Z
 * bits.  A repeated qubit is measured again after its earlier reset. */
int cliff_reset_record(cliff_tab *tab, const uint32_t *qubits, size_t k, uint64_t seed,
                       uint64_t circuit, uint64_t shot0, uint64_t m0, uint8_t *dev_record,
                       size_t ld, size_t col0, uint8_t *dev_random);

/* Classically conditioned Paulis: for i < k apply the Pauli paulis[i] (1 X,
 * 2 Y, 3 Z) to qubits[i] in every shot s whose record byte
 * dev_record[s * ld + cols[i]] (device memory, e.g. from
 * cliff_measure_record) is 1.  A Pauli conjugates every row to itself up to
 * sign (rows anticommuting with it flip: X flips rows with z = 1, Z rows
 * with x = 1, Y rows with x ^ z = 1), so the shots keep one set of X/Z bits
 * and only their sign columns differ.  Only enqueues work.  EINVAL on a bad
 * qubit, Pauli or column (cols[i] >= ld). */
int cliff_apply_cond_paulis(cliff_tab *tab, const uint32_t *qubits, const uint8_t *paulis,
                            const uint32_t *cols, size_t k, const uint8_t *dev_record, size_t ld);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  Same
 * arguments, results and error codes as cliff_measure_record (outcomes into
 * the caller's device record, bit for bit the same), but the call allocates
 * nothing and stages nothing through the context: the qubit list and the
 * register-resident pass's chunk scratch live in a static device array of
 * CLIFF_NOALLOC_SCRATCH_BYTES that the library keeps on each GPU it runs on
 * until the process ends (its chunks are as large as fits there, 48
 * measurements at n = 10,000, and it does not take the blocked pass, where
 * cliff_measure_record takes chunks of 2048, so large n run slower than with
 * cliff_measure_record).  Every call on a GPU uses that GPU's one array:
 * calls that overlap on one GPU (several host threads, or contexts on
 * different streams) race and must be serialized by the caller.
 * CLIFF_EINVAL as cliff_measure_record and while kernel timing
 * (cliff_ctx_profile) is on; CLIFF_ENOMEM if a tableau shape needed more
 * than the array (none of n <= 10,240 does). */
#define CLIFF_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int cliff_measure_record_noalloc(cliff_tab *tab, const uint32_t *qubits, size_t k, uint64_t seed,
                                 uint64_t circuit, uint64_t shot0, uint64_t m0, uint8_t *dev_record,
                                 size_t ld, size_t col0, uint8_t *dev_random);

/* Asynchronous form of cliff_measure for k <= n measurements: only enqueues
 * the work on the context stream.  The outcomes stay in the tableau's device
 * staging until cliff_tab_read_outcomes (same k, same layout as cliff_measure,
 * synchronizes the stream) or the next measurement on this tableau. */
int cliff_measure_async(cliff_tab *tab, const uint32_t *qubits, size_t k, uint64_t seed,
                        uint64_t circuit, uint64_t shot0, uint64_t m0);
int cliff_tab_read_outcomes(cliff_tab *tab, size_t k, uint8_t *host_out, uint8_t *host_random);

/* Sampling without disturbing the state: copy `tab` into `work` (bound with
 * the same n and at least `shots` sign columns; every sign column of work
 * starts as sign column 0 of tab) and measure qubits[0..k) on `work`.  `tab`
 * is left unchanged.  Output as for cliff_measure. */
int cliff_sample(cliff_tab *tab, cliff_tab *work, const uint32_t *qubits, size_t k,
                 uint64_t seed, uint64_t circuit, uint64_t shot0, uint8_t *host_out,
                 uint8_t *host_random);

/* Canonical byte-per-bit copy of the tableau: x, z as uint8 [2n][n] (row i,
 * column j), r as uint8 [shots][2n].  Export synchronizes. */
int cliff_tab_export(cliff_tab *tab, uint8_t *x, uint8_t *z, uint8_t *r);
int cliff_tab_import(cliff_tab *tab, const uint8_t *x, const uint8_t *z, const uint8_t *r);

/* Rows rows[0..k) (each < 2n, any order, repeats allowed) in the same
 * byte-per-bit form: x, z as uint8 [k][n], r as uint8 [shots][k] (nullable).
 * Copies only the 64-row words holding them, so rows of tableaux too large to
 * export whole can be checked.  Synchronizes; CLIFF_EINVAL for a row >= 2n. */
int cliff_tab_export_rows(cliff_tab *tab, const uint32_t *rows, size_t k, uint8_t *x, uint8_t *z, uint8_t *r);

/* Device-side consistency counters since bind: number of rowsums whose phase
 * came out odd on a row that should commute with the pivot (must stay 0). */
int cliff_tab_anomalies(cliff_tab *tab, uint64_t *count);

/* Counters since init/reset: out4[0] anomalies (as above), out4[1] random
 * measurements, out4[2] deterministic measurements, out4[3] algorithmic bytes
 * of the measurements: per random measurement 8 W (2 s + s_x + s_z + 3) + 80 n
 * (x and z words of the s columns where the pivot row is not I read, the s_x
 * x-words and s_z z-words written, the update mask and two counter planes;
 * the pivot-row gather and the rewrite of rows p-n and p), per deterministic
 * one 8 n W (the stabilizer half of every column read); W = ceil(2n / 64).
 * Synchronizes. */
int cliff_tab_counters(cliff_tab *tab, uint64_t *out4);
int cliff_tab_reset_counters(cliff_tab *tab);

/* Kernel timing (tracing aid): when enabled, every kernel launch made through
 * the context is bracketed by HIP events on its stream.  Kinds: 0 gate sweep,
 * 1 pivot select, 2 rowsum sweep, 3 finalize, 4 other (init/fold/copy),
 * 5 batched circuits, 6 blocked measurement pass (its x/z kernel).  Enabling (or disabling) resets the totals; reading
 * synchronizes and returns total milliseconds and launch count of a kind. */
int cliff_ctx_profile(cliff_ctx *ctx, int enable);
int cliff_ctx_profile_read(cliff_ctx *ctx, int kind, double *ms, uint64_t *launches);

/* ------------------------------------------------------------ batching ---
 * Thousands of independent small circuits in one persistent launch (the
 * phase-space method of Sec. 2 applied per circuit, each circuit held in the
 * LDS of one workgroup).  Circuit i is described by descs[i]: n qubits
 * (1 <= n <= maxn of the launch), `depth` layers whose encoded ops (see
 * cliff_encode_layers) start at word ops_off of dev_ops, with the layer
 * boundaries offs[offs_off .. offs_off+depth] (relative to ops_off; the ops
 * of one layer act on distinct qubits, as cliff_encode_layers emits them), `shots`
 * sign columns (1..64), and outcomes written as uint8 [shots][n] at byte
 * out_off of dev_out after measuring qubits 0..n-1 in order (measurement index
 * m = qubit, shot index 0..shots-1, circuit index circuit_id for the random
 * bit).  Workgroups take circuits in the order dev_order[0..count) from a
 * device queue.  team: threads per circuit, 64, 128, 256, 512 or 1024.
 * maxn (1..256) and max_shots (1..64) size each workgroup's LDS, about
 * 16 maxn ceil(2 maxn / 64) + 8 ceil(2 maxn / 64) max_shots bytes: a
 * descriptor with n > maxn or shots > max_shots is skipped and counted as
 * rejected, and the smaller the bounds, the more circuits run side by side on
 * a compute unit.  dev_work: cliff_batch_work_bytes() bytes of device scratch,
 * reset by the launch.  All pointers are device pointers; nothing is copied
 * to the host and the call only enqueues work.  CLIFF_EINVAL for a team,
 * maxn or max_shots out of range. */
typedef struct {
    uint32_t n, depth, shots, reserved;
    uint64_t ops_off, offs_off, out_off, circuit_id;
} cliff_batch_desc;

size_t cliff_batch_work_bytes(void);
int cliff_batch_run(cliff_ctx *ctx, const cliff_batch_desc *dev_descs, const uint64_t *dev_ops,
                    const uint32_t *dev_offs, uint8_t *dev_out, const uint32_t *dev_order,
                    uint32_t count, uint64_t seed, void *dev_work, uint32_t team, uint32_t maxn,
                    uint32_t max_shots);
/* Reorders, in place in host memory, the ops of every layer of one circuit's
 * encoded stream (ops as from cliff_encode_layers, layer l = ops[offs[l] ..
 * offs[l+1]), depth layers, n qubits, 1 <= n <= 256) for the batch kernel's
 * LDS banks: the ops of a layer act on distinct qubits and commute, so any
 * order gives the same state, outcomes and signs; this one spreads the column
 * accesses that the kernel issues together over distinct LDS banks.
 * Deterministic.  CLIFF_EINVAL on n out of range, NULL pointers (ops may be
 * NULL for an empty stream) or decreasing offsets. */
int cliff_batch_order_ops(uint32_t n, uint64_t *ops, const uint32_t *offs, uint32_t depth);
/* out2[0] = descriptors rejected (n or shots out of range), out2[1] = device
 * consistency-check failures, of the last launch using dev_work.  Synchronizes. */
int cliff_batch_status(cliff_ctx *ctx, const void *dev_work, uint64_t *out2);

/* --------------------------------------------------------------- graphs ---
 * Capture everything the context enqueues between begin and end into a HIP
 * graph, replayable with cliff_graph_launch on the same stream.  The context
 * must use a non-default stream.  Captured work must not change shape between
 * replays (the same pointers and sizes are reused). */
typedef struct cliff_graph cliff_graph;
int cliff_graph_begin(cliff_ctx *ctx);
int cliff_graph_end(cliff_ctx *ctx, cliff_graph **out);
int cliff_graph_launch(cliff_graph *graph);
int cliff_graph_destroy(cliff_graph *graph);

#ifdef __cplusplus
}
#endif
#endif /* CLIFF_H */
