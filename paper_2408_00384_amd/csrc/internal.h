// Internal layout and launch helpers of the tableau library (not part of the ABI).
//
// HBM layout of one tableau (all regions 256-byte aligned, inside the caller's
// buffer):
//   X, Z   : n columns x Wp words (uint64); word w of column j = rows 64w..64w+63
//            of qubit j, LSB = lowest row.  Column-major so a gate or a rowsum
//            sweep over one column is a contiguous, coalesced word stream.
//   R      : Wp x S words; R[w*S + s] = sign bits of rows 64w.. for shot s.
//   P      : Wp words of sign flips from gates not yet folded into R (gates
//            act identically on every shot, so they write one plane only).
//   scratch: snapshots of measured columns, pivot ring, pivot signs, per-
//            workgroup counter partials of two consecutive measurements,
//            deterministic-outcome accumulators, state words, outcome staging.
// The register-resident measurement's chunk scratch (persist_scratch_layout)
// is not part of a tableau: it belongs to the context that runs the pass.
// Padding rows 2n..64W-1 and padding words W..Wp-1 are always zero.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>
#include "gate_ops.h"

namespace cliff {

// Workgroup barrier ordering LDS only, for kernels whose waves share data
// through LDS alone (global memory is read or written per thread, or
// exchanged between workgroups with atomics): global loads and stores may
// stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint32_t kStateWords = 64;   // uint32 words of measurement state

// Measurement-state word indices (uint32).
enum : uint32_t {
  ST_PIVOT = 0,      // pivot row p, or kNone when deterministic
  ST_ANOMALY = 1,    // count of rows whose phase counter came out odd
  ST_DET_PAR = 2,    // deterministic branch: XOR of per-column pair parities
  ST_DET_Y = 3,      // deterministic branch: count of Y entries in the product rows
  ST_ERROR = 4,      // sticky error bits
  ST_RANDOM_CNT = 5, // random measurements since bind
  ST_DET_CNT = 6,    // deterministic measurements since bind
  ST_SUPPORT = 8,      // uint64 (words 8..9): sum over random measurements of 2 s + s_x + s_z
};

// Kernel classes timed by the profiler.
enum ProfKind : int { PK_GATE = 0, PK_SELECT, PK_SWEEP, PK_FINAL, PK_OTHER, PK_BATCH, PK_BLOCKED, kProfKinds };

// Optional hipEvent timing of kernel launches, per kernel class: events are
// recorded on the launch stream right before and after each launch and
// resolved on demand (defined in api.hip).
struct Profiler {
  bool on = false;
  struct Rec {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<hipEvent_t> pool;
  std::vector<Rec> pending;
  hipEvent_t open_ev = nullptr;
  double ms[kProfKinds] = {};
  unsigned long long launches[kProfKinds] = {};
  void begin(int kind, hipStream_t st);
  void end(int kind, hipStream_t st);
  hipError_t resolve();
  void reset();
  ~Profiler();
};


struct Dims {
  uint32_t n, S;   // qubits, shot sign columns
  uint32_t W;      // ceil(2n / 64) row words
  uint32_t Wp;     // W rounded up to 8 (column stride in words)
  uint32_t NW;     // ceil(n / 64) words of a packed row
  uint32_t SW;     // ceil(S / 64) words of packed per-shot bits
};

struct Offsets {
  size_t X, Z, R, P, M, xp, zp, rp, part, state, out, kind;
  size_t SN, piv, rps, detpar, detY, detr;
  size_t abort_flag, total;
};

// Device view passed by value to kernels.
struct TabDev {
  uint64_t *X, *Z, *R, *P;
  uint64_t *M, *xp, *zp, *rp, *part;
  uint32_t *state;
  uint8_t *out, *kind;
  uint64_t *SN;              // 3 x Wp: snapshots of the measured columns
  uint32_t *piv;             // 4: pivot rows of consecutive measurements
  uint64_t *rps;             // 2 x SW: pivot-row signs handed to the next step
  uint32_t *detpar, *detY;   // n: deterministic-outcome accumulators
  uint64_t *detr;            // n x SW
  // register-resident path (n <= 10240), per chunk of measurements: measured
  // columns and pivots, the tagged publication slots, per-workgroup counter
  // partials, and the reduced sign corrections (the chunk scratch, set for
  // each pass from persist_scratch_layout; null otherwise)
  uint64_t *SNall, *C1all, *ring, *pub;
  uint32_t *pivall, *abort_flag;
  uint32_t n, S, W, Wp, NW, SW;
};

constexpr uint32_t kPersistMaxGroups = 256;
constexpr uint32_t kPersistMaxChunk = 2048;   // measurements per chunk (qubit list held in LDS)
constexpr uint32_t kPersistMaxWp = 320;       // row words: at most 5 per lane of a wave
inline bool persist_layout(uint32_t n) {
  return n >= 1 && (2 * n + 63) / 64 <= kPersistMaxWp;
}
// Measurements per chunk of the register-resident path.  Every chunk costs
// about 50 us of fixed work (setup kernel, cooperative launch, hand-offs
// between the two streams), and only the last chunk's finalize (about 1.2 us
// per measurement) is not hidden behind a later chunk, so below n = 8192 the
// size follows sqrt(42 n) (the largest power of two up to sqrt(48 n)).  It is
// bounded by the HBM kept for per-workgroup counter partials: 1 GB for
// n >= 8192 (where the chunk is as large as that allows), else 256 MB.  With
// the blocked pass (whose chunks cost about 150 us each at n = 10,000 and
// whose finalize is about 0.25 us per measurement) n >= 3000 takes 2.5 GiB:
// 2048 measurements per chunk up to the largest n, faster from n = 3,000 on
// dense and shallow circuits alike; at n = 2,100 shallow circuits, whose
// chunks mostly run per measurement, were slower with them.
constexpr uint32_t kBlkBigChunkMinN = 3000;
inline uint32_t persist_chunk(uint32_t n, bool blocked = false) {
  const uint32_t Wp = (((2 * n + 63) / 64) + 7) & ~7u;
  const bool big = blocked && n >= kBlkBigChunkMinN;
  const size_t budget = big ? (size_t(5) << 29) : n >= 8192 ? (size_t(1) << 30) : (size_t(256) << 20);
  size_t kc = budget / (size_t(kPersistMaxGroups) * Wp * 16);
  if (n < 8192 && !big) {
    size_t target = 16;
    while (4 * target * target <= size_t(48) * n) target *= 2;
    if (kc > target) kc = target;
  }
  if (kc < 16) kc = 16;
  if (kc > kPersistMaxChunk) kc = kPersistMaxChunk;
  if (kc > n) kc = n;
  return uint32_t(kc);
}

// Largest supported qubit count (pivot bits of a workgroup's columns in LDS).
constexpr uint32_t kMaxQubits = 1u << 20;

// Launch shape of the per-measurement step kernel for n qubits.
inline uint32_t step_grid(uint32_t n) {
  uint32_t g = (n + 31) / 32;
  if (g > 256) g = 256;
  return g < 1 ? 1 : g;
}
inline uint32_t step_block(uint32_t n) { return n >= 2048 ? 1024u : 256u; }

inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

inline Dims make_dims(uint32_t n, uint32_t S) {
  Dims d;
  d.n = n;
  d.S = S;
  d.W = (2 * n + 63) / 64;
  d.Wp = (d.W + 7) & ~7u;
  d.NW = (n + 63) / 64;
  d.SW = (S + 63) / 64;
  return d;
}

inline Offsets make_offsets(const Dims &d) {
  Offsets o;
  size_t cur = 0;
  auto take = [&](size_t bytes) { size_t at = cur; cur = align256(cur + bytes); return at; };
  const size_t col = size_t(d.n) * d.Wp * 8;
  o.X = take(col);
  o.Z = take(col);
  o.R = take(size_t(d.Wp) * d.S * 8);
  o.P = take(size_t(d.Wp) * 8);
  o.M = take(size_t(d.Wp) * 8);
  o.xp = take(size_t(d.NW) * 8);
  o.zp = take(size_t(d.NW) * 8);
  o.rp = take(size_t(d.SW) * 8);
  o.part = take(2 * size_t(step_grid(d.n)) * d.Wp * 16);   // partials of two steps
  o.state = take(kStateWords * 4);
  o.out = take(size_t(d.n) * d.S);   // staging for up to n measurements per pass
  o.kind = take(size_t(d.n));
  o.SN = take(3 * size_t(d.Wp) * 8);
  o.piv = take(4 * 4);
  o.rps = take(2 * size_t(d.SW) * 8);
  o.detpar = take(size_t(d.n) * 4);
  o.detY = take(size_t(d.n) * 4);
  o.detr = take(size_t(d.n) * d.SW * 8);
  o.abort_flag = take(4);   // every layout: the init and copy kernels clear it
  o.total = cur;
  return o;
}

// Chunk scratch of the register-resident measurement for a tableau shape and
// kc measurements per chunk, two sets (chunk c and chunk c + 1 in flight
// together), offsets from a 256-byte aligned base.
struct PersistScratchLayout {
  size_t SNall, pivall, pub, C1all, ring, total;
};
inline PersistScratchLayout persist_scratch_layout(const Dims &d, uint32_t kc) {
  PersistScratchLayout o;
  size_t cur = 0;
  auto take = [&](size_t bytes) { size_t at = cur; cur = align256(cur + bytes); return at; };
  const size_t k2 = 2 * size_t(kc);
  o.SNall = take(k2 * d.Wp * 8);
  o.pivall = take(k2 * 4);
  o.pub = take(k2 * 2 * d.Wp * 8);   // [m][word][2] tagged 32-bit halves
  o.C1all = take(k2 * d.Wp * 8);
  o.ring = take(k2 * kPersistMaxGroups * d.Wp * 16);   // partials [m][workgroup][word][2]
  o.total = cur;
  return o;
}
// Point a tableau view's chunk-scratch fields into `base` (layout above).
inline void persist_scratch_bind(TabDev &t, const Dims &d, uint32_t kc, uint8_t *base) {
  const PersistScratchLayout o = persist_scratch_layout(d, kc);
  t.SNall = reinterpret_cast<uint64_t *>(base + o.SNall);
  t.pivall = reinterpret_cast<uint32_t *>(base + o.pivall);
  t.pub = reinterpret_cast<uint64_t *>(base + o.pub);
  t.C1all = reinterpret_cast<uint64_t *>(base + o.C1all);
  t.ring = reinterpret_cast<uint64_t *>(base + o.ring);
}


// Blocked pass over a chunk's random measurements (measure_block.hip): blocks
// of up to kBlkK measurements, each applied to the register-held tableau as
// one low-rank update.  Per chunk: the block's measured columns handed to the
// planner, U and the pivots of every block, per-workgroup sign partials, the
// reduced sign flips, and four counters (columns published, blocks planned,
// measurements done by the pass, columns handed over through the second
// buffer).
constexpr uint32_t kBlkK = 32;
// Smallest n for which the automatic measurement mode takes the blocked pass.
constexpr uint32_t kBlkAutoMinN = 2048;
struct BlkDev {
  uint64_t *cols;    // [2][kBlkK][Wp] measured columns of blocks to plan (block c in buffer c mod 2)
  uint64_t *U;       // [NB][kBlkK][Wp] U columns (rows that absorbed pivot t)
  uint64_t *part;    // [NB][G][3][Wp] per workgroup: (Y_old - Y_new) mod 4 (two planes), z.x parity
  uint64_t *H;       // [NB][Wp] sign flips of the block's kept and replaced rows
  uint32_t *piv;     // [NB][kBlkK] pivot rows
  uint32_t *rowu;    // [NB][kBlkK] pivots absorbed by the pivot row at its step
  uint32_t *qrow;    // [NB][kBlkK] replaced rows p_t - n
  uint32_t *rq;      // [NB][kBlkK] their bits of U (bit i: U column i)
  uint32_t *ppart;   // [NB][G][2 + kBlkK] per workgroup: pivot Y counts (two planes), Gram rows
  uint32_t *nb;      // [NB] measurements of each block (0: none)
  uint32_t *sync;    // [4] counters
  uint32_t NB;
};
struct BlkArgs {
  const uint32_t *qubits;   // device, this chunk's k entries
  uint32_t k, G;
  uint32_t abort_at;        // as for the per-measurement kernels (kNone: never)
};
struct BlkScratchLayout {
  size_t cols, U, part, H, piv, rowu, qrow, rq, ppart, nb, sync, total;
};
inline BlkScratchLayout blk_scratch_layout(const Dims &d, uint32_t kc, uint32_t G) {
  BlkScratchLayout o;
  size_t cur = 0;
  auto take = [&](size_t bytes) { size_t at = cur; cur = align256(cur + bytes); return at; };
  const size_t NB = (size_t(kc) + kBlkK - 1) / kBlkK;
  o.cols = take(2 * size_t(kBlkK) * d.Wp * 8);
  o.U = take(NB * kBlkK * d.Wp * 8);
  o.part = take(NB * G * 3 * d.Wp * 8);
  o.H = take(NB * d.Wp * 8);
  o.piv = take(NB * kBlkK * 4);
  o.rowu = take(NB * kBlkK * 4);
  o.qrow = take(NB * kBlkK * 4);
  o.rq = take(NB * kBlkK * 4);
  o.ppart = take(NB * G * (2 + kBlkK) * 4);
  o.nb = take(NB * 4);
  o.sync = take(16);
  o.total = cur;
  return o;
}
inline BlkDev blk_scratch_bind(const Dims &d, uint32_t kc, uint32_t G, uint8_t *base) {
  const BlkScratchLayout o = blk_scratch_layout(d, kc, G);
  BlkDev s;
  s.cols = reinterpret_cast<uint64_t *>(base + o.cols);
  s.U = reinterpret_cast<uint64_t *>(base + o.U);
  s.part = reinterpret_cast<uint64_t *>(base + o.part);
  s.H = reinterpret_cast<uint64_t *>(base + o.H);
  s.piv = reinterpret_cast<uint32_t *>(base + o.piv);
  s.rowu = reinterpret_cast<uint32_t *>(base + o.rowu);
  s.qrow = reinterpret_cast<uint32_t *>(base + o.qrow);
  s.rq = reinterpret_cast<uint32_t *>(base + o.rq);
  s.ppart = reinterpret_cast<uint32_t *>(base + o.ppart);
  s.nb = reinterpret_cast<uint32_t *>(base + o.nb);
  s.sync = reinterpret_cast<uint32_t *>(base + o.sync);
  s.NB = uint32_t((size_t(kc) + kBlkK - 1) / kBlkK);
  return s;
}


// ---- launchers (each defined in the .hip file holding its kernels) ----------
hipError_t launch_init_zero(const TabDev &t, hipStream_t st);
hipError_t launch_fold_pending(const TabDev &t, hipStream_t st);
hipError_t launch_gate_layer(const TabDev &t, const uint64_t *ops, uint32_t nops, hipStream_t st);
// LDS budget of the fused all-layers gate kernel (8 bytes per qubit).
constexpr size_t kFusedGateLds = 160 * 1024 - 1024;
bool fused_gates_fit(uint32_t n);
// One tableau of a many-tableau gate launch (device memory).
struct ManyDesc {
  uint64_t *X, *Z, *P;
  const uint64_t *ops;      // encoded ops of this tableau
  const uint32_t *offs;     // its layer boundaries [depth + 1]
  uint32_t n, Wp, depth, pad;
};
static_assert(sizeof(ManyDesc) == 56, "descriptor layout");
bool many_gates_fit(uint32_t max_n, uint32_t rows);
hipError_t launch_record(const TabDev &t, uint32_t cnt, uint8_t *rec, size_t ld, size_t col0, uint8_t *rnd,
                         hipStream_t st);
hipError_t launch_cond_pauli(const TabDev &t, const uint64_t *ops, uint32_t k, const uint8_t *rec, size_t ld,
                             hipStream_t st);
hipError_t launch_gates_many(const ManyDesc *dev_descs, uint32_t count, uint32_t max_n, uint32_t rows,
                             hipStream_t st);
hipError_t launch_gates_fused(const TabDev &t, const uint64_t *ops, const uint32_t *dev_offs,
                              uint32_t depth, hipStream_t st);
hipError_t launch_measure_list(const TabDev &t, const uint32_t *qubits, uint32_t k, uint64_t seed,
                               uint64_t circuit, uint64_t shot0, uint64_t m0, hipStream_t st,
                               Profiler *prof);
hipError_t launch_clear_state(const TabDev &t, hipStream_t st);
bool persist_shape(uint32_t n, uint32_t num_cus, uint32_t *G, uint32_t *L, uint32_t *CW);
// Blocked pass: G sweeper workgroups (plus one planner) and L row words per
// lane for n qubits (false = not usable on num_cus compute units).
bool blk_shape(uint32_t n, uint32_t num_cus, uint32_t *G, uint32_t *L);
// One chunk of cnt measurements: the blocked pass (it stops at the first
// deterministic measurement and leaves the count done in s.sync[2]), then
// its sign finalize (on the stream that finalizes the chunk).
hipError_t launch_blk_chunk(const TabDev &t, const BlkDev &s, const uint32_t *dev_qubits, uint32_t cnt,
                            uint32_t G, uint32_t L, uint32_t abort_at, hipStream_t st);
hipError_t launch_blk_finalize(const TabDev &t, const BlkDev &s, uint32_t cnt, uint32_t base, uint64_t seed,
                               uint64_t circuit, uint64_t shot0, uint64_t m0, uint32_t G, hipStream_t st);
// Streams and events of the register-resident path: chunk c's x/z kernel
// runs on `main` while chunk c - 1's reduction and sign walk run on `aux`;
// ev[0..1] mark x/z done and ev[2..3] finalize done per scratch buffer.
// ev[b]: chunk of scratch set b enqueued on main; ev[2 + b]: its finalize
// done on aux; ev[4 + b]: its blocked pass done on main.
struct PersistStreams {
  hipStream_t main, aux;
  hipEvent_t ev[6];
};
// *done = measurements whose launches were all enqueued (chunks before a failure).
// t carries the chunk scratch for chunks of kc measurements (persist_scratch_bind).
// blk: null, or two scratch sets of the blocked pass (blk_scratch_bind for kc
// and blk_G) that then takes each chunk's leading random measurements with
// the launch shape (blk_G, blk_L) of blk_shape.
hipError_t launch_measure_persist(const TabDev &t, uint32_t kc, const uint32_t *dev_qubits, uint32_t k,
                                  uint64_t seed, uint64_t circuit, uint64_t shot0, uint64_t m0,
                                  int num_cus, const PersistStreams &ps, Profiler *prof, uint32_t *done,
                                  uint64_t abort_at, const BlkDev *blk = nullptr, uint32_t blk_G = 0,
                                  uint32_t blk_L = 0);
// Batched circuits: team in {64, 128, 256, 512, 1024}, 1 <= maxn <= kBatchMaxN,
// 1 <= max_shots <= 64 (hipErrorInvalidValue otherwise).
constexpr uint32_t kBatchMaxN = 256;
// Reorders the ops of every layer (host memory, in place) for the batch
// kernel's LDS banks; -1 on n outside 1..kBatchMaxN, NULL or decreasing offsets.
int batch_order_ops(uint32_t n, uint64_t *ops, const uint32_t *offs, uint32_t depth);
hipError_t launch_batch(const void *descs, const uint64_t *ops, const uint32_t *offs, uint8_t *out,
                        const uint32_t *order, uint32_t count, uint64_t seed, uint32_t *work,
                        uint32_t team, uint32_t maxn, uint32_t max_shots, int num_cus, hipStream_t st);
hipError_t launch_copy_tab(const TabDev &dst, const TabDev &src, hipStream_t st);
// count words from host memory to device memory dst through kernel arguments.
hipError_t launch_store_words(uint32_t *dst, const uint32_t *host, uint32_t count, hipStream_t st);
hipError_t launch_calibrate(int kind, int num_cus, uint32_t iters, uint32_t *sink, hipStream_t st, double *work);

}  // namespace cliff
