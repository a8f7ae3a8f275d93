// Blocked measurement: a run of random Z-measurements applied to a tableau
// held in registers as one low-rank update per block of up to 32
// measurements, instead of one rowsum sweep (and one hand-off between
// workgroups) per measurement.
//
// Method: paper Sec. 2 (Aaronson & Gottesman 2004 tableau rules); outcomes,
// tableau bits and signs are those of the step-by-step rule.
//
//  * A random measurement of qubit a with pivot p (smallest stabilizer row
//    with x = 1 on column a) multiplies every other row with x = 1 on column
//    a by row p, copies row p into row p - n and sets row p to Z_a with the
//    outcome as sign.  On the bits of each column this is linear in the rows,
//    the same map for every column.  Composed over a block of measurements
//    with pivots p_0 .. p_{k-1}, every row i that is not a pivot row ends as
//        new_i = [i not replaced] old_i  XOR  sum_t U[i][t] old_{p_t},
//    old = the rows at the block's start, the replaced rows being p_t - n
//    (their old contents are dropped), and each pivot row p_t ends as Z_{a_t}.
//    The planner builds U (2n x k bits, bit-sliced: U column t over all row
//    words) from the block's measured columns alone, one measurement after
//    the other; then every column takes a single update (the sweep):
//        x ^= sum over t with x[p_t] = 1 of U_t,  same for z.
//  * Signs.  Every product formed is of commuting Pauli rows, so a final row
//    is the product of its factors (old_i if kept, and the pivot rows in
//    U[i]) in any order, and its sign is
//        sum of the factors' signs + (sum of the factors' Y counts
//        - Y count of the result) / 2 + sum over factor pairs a < b of
//        z(a).x(b)   (mod 2),
//    Y count = number of columns with x = z = 1 (i^(x.z) X^x Z^z is the
//    Hermitian Pauli of (x, z)).  With old_i taken first, the pair sum is
//    z(old_i).(x_new_i ^ x_old_i) plus the pivot rows' Gram matrix
//    G[a][b] = z(old_{p_a}).x(old_{p_b}) over the pairs in U[i].  The sweep
//    sums per row (Y_old - Y_new) mod 4 and the z.x parity, and per pivot
//    its Y count and its Gram row; the finalize kernels add them up and
//    apply the signs, a GF(2) product per shot like the x/z update.
//  * A deterministic measurement ends the blocked pass of its chunk: the
//    count done here is left in device memory, and the per-measurement
//    kernels of measure_persist.hip take the chunk's other measurements from
//    there without a host round trip.
//
// Launch: G sweeper workgroups own the columns as in measure_persist.hip
// (workgroup g the columns g (mod G), 8 waves, L whole columns of L row
// words per lane per wave, x and z in registers) plus one planner workgroup
// (one row word per thread, the block's columns and U in registers).  The
// owners of block c's measured columns hand them over during the sweep of
// block c - 2 (plain stores, a release fence, a counter; two buffers
// alternate), updated to before block c - 1; the planner, having published
// U of block c - 1 the same way, applies that U to them itself and plans
// block c at once, while each sweeper workgroup stages the published U in
// LDS and applies it to its columns.  Every wait is bounded and watches the
// tableau's abort flag.
#include <utility>

#include "internal.h"
#include "philox.h"

namespace cliff {

namespace {

constexpr uint32_t kBlkSpinLimit = 1u << 20;
constexpr uint32_t kBlkWaves = 8;
constexpr uint32_t kBlkThreads = kBlkWaves * 64;
constexpr uint32_t kBlkSignThreads = 256;

__device__ __forceinline__ uint64_t bbit(uint32_t b) { return 1ull << (b & 63); }

// Loads of data another workgroup published (coherent across the chip's L2
// slices without invalidating them): each is issued after the counter that
// announced the data was seen.
__device__ __forceinline__ uint32_t blk_ld(const uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t blk_ld64(const uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until *ctr >= target; false when the wait gave up (the abort flag is
// then raised) or the flag was already raised.
__device__ __forceinline__ bool blk_wait(const uint32_t *ctr, uint32_t target, uint32_t *abort_flag) {
  uint32_t spins = 0;
  while (blk_ld(ctr) < target) {
    if (blk_ld(abort_flag)) return false;
    if (++spins > kBlkSpinLimit) {
      atomicOr(abort_flag, 1u);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  return !blk_ld(abort_flag);
}

__device__ __forceinline__ void fence_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }

// Smallest stabilizer row with x = 1 in word w (value v) of a column, or kNone.
__device__ __forceinline__ uint32_t blk_candidate(uint64_t v, uint32_t w, uint32_t n, uint32_t W) {
  if (w >= W || w < (n >> 6)) return kNone;
  if (w == (n >> 6)) v &= ~0ull << (n & 63);
  return v ? w * 64 + uint32_t(__builtin_ctzll(v)) : kNone;
}

struct BlkShared {
  uint64_t K[kPersistMaxWp];                     // rows p_t and p_t - n of the block
  unsigned long long E0[kPersistMaxWp], E1[kPersistMaxWp], ZX[kPersistMaxWp];
  uint32_t own[kPersistMaxChunk];                // owner of each measured column: g << 8 | wave << 4 | slot
  uint32_t P[kBlkK], RU[kBlkK], gam[kBlkK], ycnt[kBlkK];
  alignas(16) uint32_t V[kBlkK];   // planner: the next block's columns' bits at this block's pivot rows
  unsigned long long best[3];   // planner: smallest offer (pivot << 32 | its bits), by step mod 3
  uint32_t abort;
};

// ---------------------------------------------------------------- planner --
// Each thread holds one row word w (plan_group below) of the block's columns
// and of U in one array, split in 32-bit halves (lo: rows 64 w .. 64 w + 31),
// threads past the last word nothing: element i is column
// a_i while measurement i is to come and U column i once it is done (the
// column becomes its own U column: M = the rows with x = 1 on it, less p and
// p - n, plus row p - n).  Measurement t with pivot p:
//   rows in M absorb row p: element i ^= M for every i whose bit p is set
//   (U columns: the pivots row p had absorbed; columns: x[p] there);
//   row p - n takes row p's bits, row p is cleared.
// One workgroup barrier per measurement: each wave offers its smallest
// candidate row together with that row's bits of every element, and every
// thread takes the smallest offer (one LDS atomic-min on pivot << 32 | its
// bits).  The 32 steps are instantiated one by one (a template per step) so
// that element indices are constants, and a step past the block's end or
// after a deterministic measurement runs with an all-zero update rather than
// leaving early (exits with the 64 element registers live made the compiler
// keep copies of them in scratch).
// Rows p - n are fixed once per block: no pivot search reads destabilizer
// rows, and no other row's update reads them, so during the block their bits
// are left as the updates make them while lane t of wave 0 tracks replaced
// row p_t - n's bits over the elements (rq) by the rule every row follows:
// at step t' its bit of element i flips when its bit of element t' is set
// and row p_t' has bit i set.
struct PlanCtx {
  uint32_t kbmax, kb, m0b, b;
  uint32_t rq, qrow;   // wave 0, lane t: replaced row p_t - n and its bits
  bool aborted, stopped;
};

// Row-word group of planner wave `wave` (thread: word 64 group + lane).  With
// five groups (W > 256, so n > 8192) waves 0 and 4 share a SIMD: they take
// groups 0 and 1, destabilizer rows only, which never search for a pivot,
// and waves 1-3 the groups that do.
__device__ __forceinline__ uint32_t plan_group(uint32_t wave, uint32_t W) {
  if (W <= 256) return wave;
  return wave == 4 ? 1u : (wave >= 1 && wave <= 3) ? wave + 1 : wave;
}

template <uint32_t D>
__device__ __forceinline__ void plan_step(uint32_t (&lo)[kBlkK], uint32_t (&hi)[kBlkK], PlanCtx &pc,
                                          const TabDev &t, const BlkDev &s, const BlkArgs &a, BlkShared &sh) {
  constexpr uint32_t tt = D;   // the block's measurement index of this step
  if (tt >= pc.kbmax) pc.stopped = true;
  const uint32_t tid = threadIdx.x, lane = tid & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const uint32_t n = t.n, W = t.W, grp = plan_group(wave, W), w = grp * 64 + lane;
  if (!pc.stopped && pc.m0b + tt == a.abort_at) {   // injected: stop as after a timed-out wait
    if (tid == 0) atomicOr(t.abort_flag, 1u);
    pc.aborted = true;
    pc.stopped = true;
  }
  const bool live = !pc.stopped;
  const uint32_t slot = tt % 3u;
  const uint32_t cl = lo[D], ch = hi[D];
  // waves past the last row word hold nothing: they only keep the barriers
  // (and leave the issue slots of their SIMD to the wave sharing it)
  const bool holds = grp * 64 < W;
  if (holds) {
    // this wave's smallest candidate and that row's bits of the elements
    const uint32_t cand = live ? blk_candidate((uint64_t(ch) << 32) | cl, w, n, W) : kNone;
    const uint64_t bal = __ballot(cand != kNone);
    uint32_t pv = kNone, rbv = 0;
    if (bal) {
      const uint32_t l = uint32_t(__builtin_ctzll(bal));
      pv = uint32_t(__builtin_amdgcn_readlane(int(cand), int(l)));
      const uint32_t sft = pv & 31;
      uint32_t v = 0;
      if (pv & 32) {
#pragma unroll
        for (uint32_t i = 0; i < kBlkK; ++i) v |= ((hi[i] >> sft) & 1u) << i;
      } else {
#pragma unroll
        for (uint32_t i = 0; i < kBlkK; ++i) v |= ((lo[i] >> sft) & 1u) << i;
      }
      rbv = uint32_t(__builtin_amdgcn_readlane(int(v), int(l)));
    }
    if (bal && lane == 0) atomicMin(&sh.best[slot], (static_cast<unsigned long long>(pv) << 32) | rbv);
  }
  // the slot of step tt + 1 was last read before this step began
  if (tid == 0) sh.best[slot == 2 ? 0 : slot + 1] = ~0ull;
  lds_barrier();
  const unsigned long long bk = sh.best[slot];
  const uint32_t p = uint32_t(bk >> 32);
  uint32_t rb = uint32_t(bk);   // row p's bits of the elements
  if (live && p == kNone) {   // deterministic: the block ends before it
    pc.kb = tt;
    pc.stopped = true;
  }
  const bool go = !pc.stopped;
  if (!go) rb = 0;
  const uint32_t wp = p >> 6, pn = p - n;
  if (go && tid == 0) {
    s.piv[size_t(pc.b) * kBlkK + tt] = p;
    s.rowu[size_t(pc.b) * kBlkK + tt] = rb & ((1u << tt) - 1u);
  }
  // rows of M absorb row p; with row p in the mask, its own bit (set exactly
  // where rb is) clears in the same XOR.  Element tt becomes U column tt: M
  // (plus row p - n, set at the block's end).
  if (holds) {
    const uint32_t bpl = go && w == wp && !(p & 32) ? 1u << (p & 31) : 0u;
    const uint32_t bph = go && w == wp && (p & 32) ? 1u << (p & 31) : 0u;
#pragma unroll
    for (uint32_t i = 0; i < kBlkK; ++i) {
      if (i == D) {
        lo[i] ^= bpl;
        hi[i] ^= bph;
      } else {
        const uint32_t msk = 0u - ((rb >> i) & 1u);
        lo[i] ^= cl & msk;
        hi[i] ^= ch & msk;
      }
    }
  }
  if (go && wave == 0) {
    const uint32_t x = rb & ~(1u << tt);
    if (lane < tt) pc.rq ^= ((pc.rq >> tt) & 1u) ? x : 0u;
    if (lane == tt) {
      pc.rq = rb | (1u << tt);
      pc.qrow = pn;
    }
  }
  // each step starts from the elements as registers (keeps the compiler from
  // carrying XOR expressions of several steps)
#pragma unroll
  for (uint32_t i = 0; i < kBlkK; ++i) asm volatile("" : "+v"(lo[i]), "+v"(hi[i]));
}

template <uint32_t... D>
__device__ __forceinline__ void plan_block(uint32_t (&lo)[kBlkK], uint32_t (&hi)[kBlkK], PlanCtx &pc,
                                           const TabDev &t, const BlkDev &s, const BlkArgs &a, BlkShared &sh,
                                           std::integer_sequence<uint32_t, D...>) {
  (plan_step<D>(lo, hi, pc, t, s, a, sh), ...);
}

// After publishing block b the planner brings block b + 1's measured columns
// (as they stood before block b, handed over by their owners during the
// sweep of block b - 1) up to date itself: x ^= sum over pivots t with
// x[p_t] = 1 of U_t, rows p_t and p_t - n set apart, a 32 x 32 GF(2) product
// per row word.  It then plans block b + 1 at once instead of waiting for the
// sweepers to update and hand over those columns.
__device__ __forceinline__ void blk_planner(const TabDev &t, const BlkDev &s, const BlkArgs &a, BlkShared &sh,
                                            uint64_t *sN, uint32_t US) {
  const uint32_t tid = threadIdx.x, lane = tid & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const uint32_t n = t.n, W = t.W, Wp = t.Wp, k = a.k, grp = plan_group(wave, W), w = grp * 64 + lane;
  PlanCtx pc;
  pc.aborted = false;
  uint32_t lo[kBlkK], hi[kBlkK];
  uint32_t cum[2] = {0u, 0u};   // columns handed over so far through each of the two buffers
  {
    const uint32_t kb0 = k < kBlkK ? k : kBlkK;
    cum[0] = kb0;
    if (tid == 0) sh.abort = blk_wait(&s.sync[0], kb0, t.abort_flag) ? 0u : 1u;
    __syncthreads();
    if (sh.abort) return;
#pragma unroll
    for (uint32_t i = 0; i < kBlkK; ++i) {
      const uint64_t v = (i < kb0 && w < W) ? blk_ld64(s.cols + size_t(i) * Wp + w) : 0ull;
      lo[i] = uint32_t(v);
      hi[i] = uint32_t(v >> 32);
    }
  }
  for (uint32_t b = 0;; ++b) {
    const uint32_t m0b = b * kBlkK;
    const uint32_t kbmax = k - m0b < kBlkK ? k - m0b : kBlkK;
    if (tid == 0) {
      sh.best[0] = ~0ull;
      sh.best[1] = ~0ull;
      sh.best[2] = ~0ull;
    }
    __syncthreads();
    pc.kbmax = kbmax;
    pc.kb = kbmax;
    pc.m0b = m0b;
    pc.b = b;
    pc.rq = 0;
    pc.qrow = 0;
    pc.stopped = false;
    plan_block(lo, hi, pc, t, s, a, sh, std::make_integer_sequence<uint32_t, kBlkK>{});
    if (pc.aborted) return;
    const uint32_t kb = pc.kb;
    if (w < W) {
#pragma unroll
      for (uint32_t i = 0; i < kBlkK; ++i)
        if (i < kb) s.U[(size_t(b) * kBlkK + i) * Wp + w] = (uint64_t(hi[i]) << 32) | lo[i];
    }
    // the replaced rows and their bits of U (the stored U has stale bits
    // there; its readers write these over them)
    if (wave == 0 && lane < kb) {
      s.qrow[size_t(b) * kBlkK + lane] = pc.qrow;
      s.rq[size_t(b) * kBlkK + lane] = pc.rq;
    }
    const uint32_t m0n = m0b + kBlkK;
    const bool last = kb < kbmax || m0n >= k;
    const uint32_t kbn = last ? 0u : (k - m0n < kBlkK ? k - m0n : kBlkK);
    const uint32_t nbuf = (b + 1) & 1u;
    // ---- block b + 1's columns, as they stood before block b (waited for
    // and loaded while the stores of U drain; all 32 loads in flight before
    // the first is used)
    if (!last) {
      cum[nbuf] += kbn;
      if (tid == 0) sh.abort = blk_wait(&s.sync[nbuf ? 3 : 0], cum[nbuf], t.abort_flag) ? 0u : 1u;
      __syncthreads();
      if (sh.abort) return;
    }
    uint32_t nl[kBlkK], nh[kBlkK];
#pragma unroll
    for (uint32_t j = 0; j < kBlkK; ++j) {
      const uint64_t v = (j < kbn && w < W) ? blk_ld64(s.cols + (size_t(nbuf) * kBlkK + j) * Wp + w) : 0ull;
      nl[j] = uint32_t(v);
      nh[j] = uint32_t(v >> 32);
    }
    fence_release();
    __syncthreads();
    if (tid == 0) {
      s.nb[b] = kb;
      if (kb < kbmax) s.sync[2] = m0b + kb;
      fence_release();
      __hip_atomic_store(&s.sync[1], b + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (last) {
      if (kb == kbmax && tid == 0) s.sync[2] = k;
      return;
    }
#pragma unroll
    for (uint32_t j = 0; j < kBlkK; ++j)
      if (w < US) sN[j * US + w] = (uint64_t(nh[j]) << 32) | nl[j];
    if (w < W) {
      sh.K[w] = 0;
      sh.ZX[w] = 0;
    }
    __syncthreads();
    // wave 0, lane t < kb: V_t = the columns' bits at pivot row p_t (bit j:
    // column j), and replaced row p_t - n: its bit of column j is the parity
    // of column j's bits at the pivots its U row holds, written over the
    // staged column; rows p_t marked in sh.K, rows p_t - n in sh.ZX
    if (wave == 0) {
      const bool mine = lane < kb;
      const uint32_t q = pc.qrow, p = q + n;
      uint32_t v = 0, oq = 0;
      if (mine) {
        // (columns past kbn are staged as zeros; the 32-bit halves holding
        // rows p and q, eight reads of each in flight at a time)
        const uint32_t *s32 = reinterpret_cast<const uint32_t *>(sN);
        const uint32_t ap = (p >> 5), aq = (q >> 5), sp = p & 31, sq = q & 31;
#pragma unroll
        for (uint32_t j = 0; j < kBlkK; ++j) {
          v |= ((s32[j * 2 * US + ap] >> sp) & 1u) << j;
          oq |= ((s32[j * 2 * US + aq] >> sq) & 1u) << j;
          if ((j & 7u) == 7u) __builtin_amdgcn_sched_barrier(0);
        }
        atomicOr(reinterpret_cast<unsigned long long *>(&sh.K[p >> 6]), (unsigned long long)bbit(p));
        atomicOr(&sh.ZX[q >> 6], (unsigned long long)bbit(q));
      }
      if (lane < kBlkK) sh.V[lane] = v;   // 0 for t >= kb
      uint32_t f = 0;
#pragma unroll
      for (uint32_t tt = 0; tt < kBlkK; ++tt) {
        const uint32_t vt = uint32_t(__builtin_amdgcn_readlane(int(v), int(tt)));
        f ^= ((pc.rq >> tt) & 1u) ? vt : 0u;
      }
      if (mine) {
        const uint32_t d = f ^ oq;
        unsigned long long *col = reinterpret_cast<unsigned long long *>(sN + (q >> 6));
        const unsigned long long m = bbit(q);
#pragma unroll
        for (uint32_t j = 0; j < kBlkK; ++j)
          if ((d >> j) & 1u) atomicXor(col + size_t(j) * US, m);
      }
    }
    __syncthreads();
    // the next block's columns brought up to date: pivot rows cleared,
    // x ^= sum over t with V_t set of U_t (U's stale replaced rows left
    // out), replaced rows taken from sN; waves past the last row word
    // hold nothing
    if (grp * 64 < W) {
      const uint64_t kq = w < W ? sh.K[w] : 0ull, qq = w < W ? uint64_t(sh.ZX[w]) : 0ull;
      const uint32_t kl = ~uint32_t(kq | qq), kh = ~uint32_t((kq | qq) >> 32), ql = ~uint32_t(qq), qh = ~uint32_t(qq >> 32);
#pragma unroll
      for (uint32_t j = 0; j < kBlkK; ++j) {
        nl[j] &= kl;
        nh[j] &= kh;
      }
      // (V_t = 0 past the block's count: those elements, not U columns,
      // drop out; V read four pivots at a time)
#pragma unroll
      for (uint32_t t4 = 0; t4 < kBlkK / 4; ++t4) {
        const uint4 v4 = reinterpret_cast<const uint4 *>(sh.V)[t4];
        const uint32_t vq[4] = {v4.x, v4.y, v4.z, v4.w};
#pragma unroll
        for (uint32_t r = 0; r < 4; ++r) {
          const uint32_t tt = 4 * t4 + r;
          const uint32_t vt = __builtin_amdgcn_readfirstlane(vq[r]);
          const uint32_t ul = lo[tt] & ql, uh = hi[tt] & qh;
#pragma unroll
          for (uint32_t j = 0; j < kBlkK; ++j) {
            const uint32_t msk = 0u - ((vt >> j) & 1u);
            nl[j] ^= ul & msk;
            nh[j] ^= uh & msk;
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (uint32_t j = 0; j < kBlkK; ++j) {
        const uint64_t f = qq ? sN[j * US + w] & qq : 0ull;
        lo[j] = nl[j] | uint32_t(f);
        hi[j] = nh[j] | uint32_t(f >> 32);
      }
    }
  }
}

// ---------------------------------------------------------------- sweeper --
template <int L>
__device__ __forceinline__ void blk_sweeper(const TabDev &t, const BlkDev &s, const BlkArgs &a, BlkShared &sh, uint64_t *sU) {
  constexpr int CW = L;
  constexpr uint32_t US = 64 * L;   // row stride of U in LDS (words)
  const uint32_t tid = threadIdx.x, lane = tid & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const uint32_t g = blockIdx.x, G = a.G, n = t.n, W = t.W, Wp = t.Wp, k = a.k;
  const uint32_t C = g < n ? (n - g + G - 1) / G : 0;
  const uint32_t ns = C > wave ? (C - wave + kBlkWaves - 1) / kBlkWaves : 0;
  const uint32_t me = (g << 8) | (wave << 4);

  uint64_t xr[CW][L], zr[CW][L];
#pragma unroll
  for (int c = 0; c < CW; ++c) {
    const uint32_t col = g + (wave + uint32_t(c) * kBlkWaves) * G;
#pragma unroll
    for (int i = 0; i < L; ++i) {
      const uint32_t w = uint32_t(i) * 64 + lane;
      const bool have = uint32_t(c) < ns && w < W;
      const size_t at = have ? size_t(col) * Wp + w : 0;
      const uint64_t xv = t.X[at], zv = t.Z[at];
      xr[c][i] = have ? xv : 0ull;
      zr[c][i] = have ? zv : 0ull;
    }
  }
  unsigned long long sup = 0;
  uint32_t done = 0;
  // this wave's columns measured in [m0, m0 + cnt), as they stand now, for
  // the planner
  auto publish_cols = [&](uint32_t m0, uint32_t cnt, uint32_t buf) {
    for (uint32_t tt = 0; tt < cnt; ++tt) {
      const uint32_t o = sh.own[m0 + tt];
      if ((o & ~15u) != me) continue;   // wave-uniform
      const uint32_t cs = o & 15u;
#pragma unroll
      for (int c = 0; c < CW; ++c) {
        if (uint32_t(c) != cs) continue;
#pragma unroll
        for (int i = 0; i < L; ++i) {
          const uint32_t w = uint32_t(i) * 64 + lane;
          if (w < W) s.cols[(size_t(buf) * kBlkK + tt) * Wp + w] = xr[c][i];
        }
      }
      fence_release();
      if (lane == 0) atomicAdd(&s.sync[buf ? 3 : 0], 1u);
    }
  };
  for (uint32_t b = 0;; ++b) {
    const uint32_t m0b = b * kBlkK;
    if (m0b >= k) break;
    const uint32_t kbmax = k - m0b < kBlkK ? k - m0b : kBlkK;
    // ---- the first two blocks' columns (later blocks' come out of the sweep
    // two blocks before, see below); block c goes through buffer c mod 2
    if (b == 0) {
      publish_cols(0, kbmax, 0);
      if (kBlkK < k) publish_cols(kBlkK, k - kBlkK < kBlkK ? k - kBlkK : kBlkK, 1);
    }
    // ---- the plan of block b
    if (tid == 0) sh.abort = blk_wait(&s.sync[1], b + 1, t.abort_flag) ? 0u : 1u;
    __syncthreads();
    if (sh.abort) return;
    // every load of the block's plan is issued before the first is used
    // (entries past the block's count are stale and never read)
    const uint32_t kb = blk_ld(s.nb + b);
    {
      uint32_t pv = 0, rv = 0;
      if (tid < kBlkK) {
        pv = blk_ld(s.piv + size_t(b) * kBlkK + tid);
        rv = blk_ld(s.rowu + size_t(b) * kBlkK + tid);
      }
      // U in passes of kPass loads per thread, all in flight together
      constexpr uint32_t kStage = (kBlkK * US + kBlkThreads - 1) / kBlkThreads, kPass = 5;
#pragma unroll
      for (uint32_t j0 = 0; j0 < kStage; j0 += kPass) {
        uint64_t tmp[kPass];
#pragma unroll
        for (uint32_t j = 0; j < kPass; ++j) {
          const uint32_t idx = tid + (j0 + j) * kBlkThreads, i = idx / US, w = idx % US;
          tmp[j] = (j0 + j < kStage && i < kBlkK && w < W) ? blk_ld64(s.U + (size_t(b) * kBlkK + i) * Wp + w) : 0ull;
        }
#pragma unroll
        for (uint32_t j = 0; j < kPass; ++j) {
          const uint32_t idx = tid + (j0 + j) * kBlkThreads;
          if (j0 + j < kStage && idx < kBlkK * US) sU[idx] = tmp[j];
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      if (tid < kBlkK) {
        sh.P[tid] = pv;
        sh.RU[tid] = rv;
        sh.gam[tid] = 0;
        sh.ycnt[tid] = 0;
      }
    }
    if (kb == 0) break;
    for (uint32_t w = tid; w < W; w += kBlkThreads) {
      sh.K[w] = 0;
      sh.E0[w] = 0;
      sh.E1[w] = 0;
      sh.ZX[w] = 0;
    }
    __syncthreads();
    for (uint32_t i = tid; i < kb; i += kBlkThreads) {
      const uint32_t p = sh.P[i], pn = p - n;
      atomicOr(reinterpret_cast<unsigned long long *>(&sh.K[p >> 6]), (unsigned long long)bbit(p));
      atomicOr(reinterpret_cast<unsigned long long *>(&sh.K[pn >> 6]), (unsigned long long)bbit(pn));
      // replaced row i: its bits of the staged U
      const uint32_t row = blk_ld(s.qrow + size_t(b) * kBlkK + i), bits = blk_ld(s.rq + size_t(b) * kBlkK + i);
      unsigned long long *col = reinterpret_cast<unsigned long long *>(sU + (row >> 6));
      const unsigned long long m = bbit(row);
      for (uint32_t j = 0; j < kb; ++j) {
        if ((bits >> j) & 1u)
          atomicOr(col + j * US, m);
        else
          atomicAnd(col + j * US, ~m);
      }
    }
    __syncthreads();
    // ---- x and z of this wave's columns at the pivot rows (bit i = pivot i):
    // lane i fetches row p_i's word from the lane holding it (a cross-lane
    // permute per slot with stabilizer rows), and ballots collect the bits
    uint32_t bx[CW], bz[CW];
    {
      const uint32_t pi = sh.P[lane < kb ? lane : 0u];
      const uint32_t wpi = pi >> 6, src = (wpi & 63u) << 2, ipi = wpi >> 6, sft = pi & 63u;
      uint32_t xb[CW], zb[CW];
#pragma unroll
      for (int c = 0; c < CW; ++c) {
        xb[c] = 0;
        zb[c] = 0;
      }
#pragma unroll
      for (int ii = 0; ii < L; ++ii) {
        if (uint32_t(ii) < ((n >> 6) >> 6)) continue;   // destabilizer words only
#pragma unroll
        for (int c = 0; c < CW; ++c) {
          const uint32_t xl = uint32_t(__builtin_amdgcn_ds_bpermute(int(src), int(uint32_t(xr[c][ii]))));
          const uint32_t xh = uint32_t(__builtin_amdgcn_ds_bpermute(int(src), int(uint32_t(xr[c][ii] >> 32))));
          const uint32_t zl = uint32_t(__builtin_amdgcn_ds_bpermute(int(src), int(uint32_t(zr[c][ii]))));
          const uint32_t zh = uint32_t(__builtin_amdgcn_ds_bpermute(int(src), int(uint32_t(zr[c][ii] >> 32))));
          const uint32_t xw = sft & 32 ? xh : xl, zw = sft & 32 ? zh : zl;
          if (ipi == uint32_t(ii)) {
            xb[c] = (xw >> (sft & 31)) & 1u;
            zb[c] = (zw >> (sft & 31)) & 1u;
          }
          // one column's permutes at a time (bounds the registers they hold)
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      const bool mine = lane < kb;
#pragma unroll
      for (int c = 0; c < CW; ++c) {
        bx[c] = uint32_t(__ballot(mine && xb[c]));
        bz[c] = uint32_t(__ballot(mine && zb[c]));
      }
    }
    // ---- Y counts of the kept rows before the update (added to the
    // workgroup's mod-4 sums in LDS: the XOR's old value gives the carry);
    // drop rows p_t, p_t - n
    uint64_t zx[L];
#pragma unroll
    for (int i = 0; i < L; ++i) {
      const uint32_t w = uint32_t(i) * 64 + lane;
      const uint64_t kw = w < W ? sh.K[w] : 0ull;
      uint64_t e0 = 0, e1 = 0;
      zx[i] = 0;
#pragma unroll
      for (int c = 0; c < CW; ++c) {
        const uint64_t y = xr[c][i] & zr[c][i] & ~kw;
        e1 ^= e0 & y;
        e0 ^= y;
        xr[c][i] &= ~kw;
        zr[c][i] &= ~kw;
      }
      if (w < W) {
        const unsigned long long old = atomicXor(&sh.E0[w], (unsigned long long)e0);
        atomicXor(&sh.E1[w], (unsigned long long)(e1 ^ (old & e0)));
      }
    }
    // ---- this wave's columns measured two blocks on: x first, and handed
    // to the planner at once (it brings them up to date with the next
    // block's update itself)
    uint32_t early = 0;
    {
      const uint32_t m0n = m0b + 2 * kBlkK;
      const uint32_t kbn = (kb == kbmax && m0n < k) ? (k - m0n < kBlkK ? k - m0n : kBlkK) : 0u;
      for (uint32_t tt = 0; tt < kbn; ++tt) {
        const uint32_t o = sh.own[m0n + tt];
        if ((o & ~15u) == me) early |= 1u << (o & 15u);
      }
      if (early) {   // wave-uniform
        for (uint32_t i = 0; i < kb; ++i) {
          uint64_t u[L];
#pragma unroll
          for (int ii = 0; ii < L; ++ii) u[ii] = sU[i * US + uint32_t(ii) * 64 + lane];
#pragma unroll
          for (int c = 0; c < CW; ++c) {
            if (((early >> c) & 1u) && ((bx[c] >> i) & 1u)) {
#pragma unroll
              for (int ii = 0; ii < L; ++ii) xr[c][ii] ^= u[ii];
            }
          }
        }
        publish_cols(m0n, kbn, b & 1u);
      }
    }
    // ---- x ^= U (x at the pivots), with the z.x parity of the kept rows
    for (uint32_t i = 0; i < kb; ++i) {
      uint64_t u[L];
#pragma unroll
      for (int ii = 0; ii < L; ++ii) u[ii] = sU[i * US + uint32_t(ii) * 64 + lane];
#pragma unroll
      for (int c = 0; c < CW; ++c) {
        if ((bx[c] >> i) & 1u) {
          const bool upd = !((early >> c) & 1u);
#pragma unroll
          for (int ii = 0; ii < L; ++ii) {
            if (upd) xr[c][ii] ^= u[ii];
            zx[ii] ^= zr[c][ii] & u[ii];
          }
        }
      }
    }
    // ---- z ^= U (z at the pivots)
    for (uint32_t i = 0; i < kb; ++i) {
      uint64_t u[L];
#pragma unroll
      for (int ii = 0; ii < L; ++ii) u[ii] = sU[i * US + uint32_t(ii) * 64 + lane];
#pragma unroll
      for (int c = 0; c < CW; ++c) {
        if ((bz[c] >> i) & 1u) {
#pragma unroll
          for (int ii = 0; ii < L; ++ii) zr[c][ii] ^= u[ii];
        }
      }
    }
    // ---- pivot rows of this wave's measured columns: z = 1 on the column
    for (uint32_t i = 0; i < kb; ++i) {
      const uint32_t o = sh.own[m0b + i];
      if ((o & ~15u) != me) continue;
      const uint32_t cs = o & 15u, p = sh.P[i], wp = p >> 6, ip = wp >> 6;
      const uint64_t bit = lane == (wp & 63) ? bbit(p) : 0ull;
#pragma unroll
      for (int c = 0; c < CW; ++c) {
        if (uint32_t(c) != cs) continue;
#pragma unroll
        for (int ii = 0; ii < L; ++ii)
          if (uint32_t(ii) == ip) zr[c][ii] |= bit;
      }
    }
    // ---- minus the Y counts after the update: count them (mod 4) and add
    // three times the count
#pragma unroll
    for (int i = 0; i < L; ++i) {
      const uint32_t w = uint32_t(i) * 64 + lane;
      uint64_t e0 = 0, e1 = 0;
#pragma unroll
      for (int c = 0; c < CW; ++c) {
        const uint64_t y = xr[c][i] & zr[c][i];
        e1 ^= e0 & y;
        e0 ^= y;
      }
      // -(e0 + 2 e1) = e0 + 2 (e1 ^ e0)  (mod 4)
      e1 ^= e0;
      if (w < W) {
        const unsigned long long old = atomicXor(&sh.E0[w], (unsigned long long)e0);
        atomicXor(&sh.E1[w], (unsigned long long)(e1 ^ (old & e0)));
        atomicXor(&sh.ZX[w], (unsigned long long)zx[i]);
      }
    }
    // ---- per pivot: Y count (mod 4), Gram row, and the support of the pivot
    // row at its step (for the device counters)
    // (lane i: pivot i)
    {
      const uint32_t la = lane & 31u;
      const uint32_t ru = lane < kb ? sh.RU[la] : 0u;
      uint32_t ycnt = 0, gacc = 0, sups = 0;
#pragma unroll
      for (int c = 0; c < CW; ++c) {
        const uint32_t bxc = bx[c], bzc = bz[c];
        ycnt += ((bxc & bzc) >> la) & 1u;
        gacc ^= ((bzc >> la) & 1u) ? bxc : 0u;
        // the pivot row at its step: row p_i plus the pivots it had absorbed
        const uint32_t xs = ((bxc >> la) ^ uint32_t(__popc(bxc & ru))) & 1u;
        const uint32_t zs = ((bzc >> la) ^ uint32_t(__popc(bzc & ru))) & 1u;
        sups += 2 * (xs | zs) + xs + zs;
      }
      if (lane < kb) {
        if (ycnt) atomicAdd(&sh.ycnt[la], ycnt);
        if (gacc) atomicXor(&sh.gam[la], gacc);
        sup += sups;
      }
    }
    // ---- store this workgroup's partials
    __syncthreads();
    uint64_t *part = s.part + (size_t(b) * G + g) * 3 * Wp;
    for (uint32_t w = tid; w < W; w += kBlkThreads) {
      part[w] = sh.E0[w];
      part[Wp + w] = sh.E1[w];
      part[2 * Wp + w] = sh.ZX[w];
    }
    uint32_t *pp = s.ppart + (size_t(b) * G + g) * (2 + kBlkK);
    if (wave == 0) {
      // pivot Y counts mod 4 as two bit planes
      const uint32_t yc = lane < kb ? sh.ycnt[lane] & 3u : 0u;
      const uint32_t y0 = uint32_t(__ballot(yc & 1u)), y1 = uint32_t(__ballot(yc & 2u));
      if (lane == 0) {
        pp[0] = y0;
        pp[1] = y1;
      }
      if (lane < kb) pp[2 + lane] = sh.gam[lane];
    }
    done += kb;
    if (kb < kbmax) break;
  }
  // ---- the tableau back to HBM
#pragma unroll
  for (int c = 0; c < CW; ++c) {
    if (uint32_t(c) >= ns) continue;
    const uint32_t col = g + (wave + uint32_t(c) * kBlkWaves) * G;
#pragma unroll
    for (int i = 0; i < L; ++i) {
      const uint32_t w = uint32_t(i) * 64 + lane;
      if (w < W) {
        t.X[size_t(col) * Wp + w] = xr[c][i];
        t.Z[size_t(col) * Wp + w] = zr[c][i];
      }
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) sup += __shfl_xor(sup, off);
  if (lane == 0 && sup) atomicAdd(reinterpret_cast<unsigned long long *>(t.state + ST_SUPPORT), sup);
  if (g == 0 && tid == 0 && done) atomicAdd(&t.state[ST_RANDOM_CNT], done);
}

template <int L>
__global__ void __launch_bounds__(kBlkThreads) k_blk(TabDev t, BlkDev s, BlkArgs a) {
  extern __shared__ uint64_t s_dynU[];
  __shared__ BlkShared sh;
  // an earlier chunk of this pass gave up: leave everything as it is
  if (__builtin_amdgcn_readfirstlane(blk_ld(t.abort_flag))) return;
  for (uint32_t m = threadIdx.x; m < a.k; m += kBlkThreads) {
    const uint32_t j = a.qubits[m], q = j / a.G;
    sh.own[m] = ((j % a.G) << 8) | ((q & 7u) << 4) | (q >> 3);
  }
  __syncthreads();
  if (blockIdx.x == a.G)
    blk_planner(t, s, a, sh, s_dynU, 64u * L);
  else
    blk_sweeper<L>(t, s, a, sh, s_dynU);
}

// The replaced rows' bits written over the stored U of every block (one
// thread per replaced row), for the finalize kernels.
__global__ void __launch_bounds__(kBlkK) k_blk_patch(TabDev t, BlkDev s) {
  const uint32_t b = blockIdx.x, q = threadIdx.x;
  if (b >= s.NB || blk_ld(t.abort_flag)) return;
  const uint32_t kb = s.nb[b];
  if (q >= kb) return;
  const uint32_t row = s.qrow[size_t(b) * kBlkK + q], bits = s.rq[size_t(b) * kBlkK + q];
  unsigned long long *col = reinterpret_cast<unsigned long long *>(s.U + size_t(b) * kBlkK * t.Wp + (row >> 6));
  const unsigned long long m = bbit(row);
  for (uint32_t j = 0; j < kb; ++j) {
    if ((bits >> j) & 1u)
      atomicOr(col + size_t(j) * t.Wp, m);
    else
      atomicAnd(col + size_t(j) * t.Wp, ~m);
  }
}

// Clear the pass counters and block counts of a chunk (kernel stores only:
// capture-safe).
__global__ void k_blk_begin(BlkDev s) {
  const uint32_t i = threadIdx.x;
  if (i < 4) s.sync[i] = 0;
  for (uint32_t b = i; b < s.NB; b += blockDim.x) s.nb[b] = 0;
}

// ---------------------------------------------------------------- reduce ---
// Per block and row word: the sign flips H = (Y_old - Y_new + sum of the
// absorbed pivots' Y counts) / 2 + z.x parity + the Gram pairs of the absorbed
// pivots (mod 2), summed over the sweeper workgroups; the low bit of the
// phase must vanish on every row but the pivot rows (counted as anomalies).
__global__ void __launch_bounds__(256) k_blk_reduce(TabDev t, BlkDev s, uint32_t G) {
  __shared__ uint32_t s_yp0, s_yp1, s_gam[kBlkK], s_P[kBlkK];
  const uint32_t b = blockIdx.x, tid = threadIdx.x;
  if (b >= s.NB) return;
  const uint32_t kb = s.nb[b];
  if (kb == 0 || blk_ld(t.abort_flag)) return;
  const uint32_t n = t.n, W = t.W, Wp = t.Wp;
  if (tid < kBlkK) s_gam[tid] = 0;
  if (tid == 0) {
    s_yp0 = 0;
    s_yp1 = 0;
  }
  if (tid < kb) s_P[tid] = s.piv[size_t(b) * kBlkK + tid];
  __syncthreads();
  // pivot partials: thread (i, q0) = (tid mod 32, tid / 32) sums Gram row i
  // (and, for i = 0, the Y-count planes) over workgroups q0, q0 + 8, ...
  {
    const uint32_t i = tid & 31u, q0 = tid >> 5, nq = blockDim.x >> 5;
    uint32_t gv = 0, y0 = 0, y1 = 0;
#pragma unroll 4
    for (uint32_t q = q0; q < G; q += nq) {
      const uint32_t *pp = s.ppart + (size_t(b) * G + q) * (2 + kBlkK);
      if (i < kb) gv ^= pp[2 + i];
      if (i == 0) {
        const uint32_t v0 = pp[0], v1 = pp[1];
        y1 ^= v1 ^ (y0 & v0);
        y0 ^= v0;
      }
    }
    if (i < kb && gv) atomicXor(&s_gam[i], gv);
    if (i == 0) {
      const uint32_t old = atomicXor(&s_yp0, y0);
      atomicXor(&s_yp1, y1 ^ (old & y0));
    }
  }
  __syncthreads();
  const uint32_t w = blockIdx.y * blockDim.x + tid;
  if (w >= W) return;
  uint64_t c0 = 0, c1 = 0, zx = 0;
  // (unrolled: the workgroups' loads in flight together)
#pragma unroll 8
  for (uint32_t q = 0; q < G; ++q) {
    const uint64_t *part = s.part + (size_t(b) * G + q) * 3 * Wp;
    const uint64_t v0 = part[w], v1 = part[Wp + w], v2 = part[2 * Wp + w];
    c1 ^= v1 ^ (c0 & v0);
    c0 ^= v0;
    zx ^= v2;
  }
  uint64_t repl = 0, cons = 0;
  for (uint32_t i = 0; i < kb; ++i) {
    const uint32_t p = s_P[i], pn = p - n;
    if ((p >> 6) == w) cons |= bbit(p);
    if ((pn >> 6) == w) repl |= bbit(pn);
  }
  const uint64_t *U = s.U + size_t(b) * kBlkK * Wp + w;
  uint64_t u[kBlkK];
#pragma unroll
  for (uint32_t i = 0; i < kBlkK; ++i) u[i] = i < kb ? U[size_t(i) * Wp] : 0ull;
  const uint32_t yp0 = s_yp0, yp1 = s_yp1;
#pragma unroll
  for (uint32_t i = 0; i < kBlkK; ++i) {
    if ((yp0 >> i) & 1u) {
      c1 ^= c0 & u[i];
      c0 ^= u[i];
    }
    if ((yp1 >> i) & 1u) c1 ^= u[i];
  }
  c1 ^= zx & ~repl;
#pragma unroll
  for (uint32_t ia = 0; ia + 1 < kBlkK; ++ia) {
    const uint32_t gm = ia + 1 < kb ? s_gam[ia] & ~((2u << ia) - 1u) : 0u;   // pairs (ia, ib > ia)
    uint64_t acc = 0;
#pragma unroll
    for (uint32_t ib = ia + 1; ib < kBlkK; ++ib)
      if ((gm >> ib) & 1u) acc ^= u[ib];
    c1 ^= u[ia] & acc;
  }
  const uint64_t odd = c0 & ~cons;
  if (odd) atomicAdd(&t.state[ST_ANOMALY], uint32_t(__popcll(odd)));
  s.H[size_t(b) * Wp + w] = c1 & ~cons;
}

// ---------------------------------------------------------------- signs ---
// One workgroup per shot walks the chunk's blocks in order with the shot's
// sign column in registers (two row words per thread):
//   r = [kept] r ^ H ^ sum over pivots t with r[p_t] = 1 of U_t,
// then the pivot rows take the outcomes (Philox bits).  Measurement i of
// block b has index base + 32 b + i in the call.
__global__ void __launch_bounds__(kBlkSignThreads) k_blk_signs(TabDev t, BlkDev s, uint32_t k, uint32_t base,
                                                               uint64_t seed, uint64_t circuit, uint64_t shot0,
                                                               uint64_t m0) {
  __shared__ uint64_t s_r[kPersistMaxWp];
  __shared__ uint32_t s_P[kBlkK], s_o, s_rp;
  const uint32_t sh = blockIdx.x, tid = threadIdx.x, lane = tid & 63, n = t.n, W = t.W, Wp = t.Wp, S = t.S;
  if (blk_ld(t.abort_flag)) return;
  uint64_t r[2];
#pragma unroll
  for (uint32_t j = 0; j < 2; ++j) {
    const uint32_t w = tid + j * kBlkSignThreads;
    r[j] = w < W ? t.R[size_t(w) * S + sh] : 0ull;
  }
  uint32_t done = 0;
  for (uint32_t b = 0; b < s.NB && b * kBlkK < k; ++b) {
    const uint32_t kb = s.nb[b];
    if (kb == 0) break;
    // this block's H and U words of the thread's two row words, all loads in
    // flight together (none depends on the signs)
    uint64_t h[2], u[2][kBlkK];
#pragma unroll
    for (uint32_t j = 0; j < 2; ++j) {
      const uint32_t w = tid + j * kBlkSignThreads;
      h[j] = w < W ? s.H[size_t(b) * Wp + w] : 0ull;
      const uint64_t *U = s.U + size_t(b) * kBlkK * Wp + w;
#pragma unroll
      for (uint32_t i = 0; i < kBlkK; ++i) u[j][i] = (i < kb && w < W) ? U[size_t(i) * Wp] : 0ull;
    }
#pragma unroll
    for (uint32_t j = 0; j < 2; ++j) {
      const uint32_t w = tid + j * kBlkSignThreads;
      if (w < W) s_r[w] = r[j];
    }
    if (tid < kb) s_P[tid] = s.piv[size_t(b) * kBlkK + tid];
    __syncthreads();
    if (tid < 64) {
      // signs of the pivot rows at the block's start; outcome bits
      const uint32_t p = tid < kb ? s_P[tid] : 0u;
      const uint64_t rp = __ballot(tid < kb && ((s_r[p >> 6] >> (p & 63)) & 1u));
      const uint32_t slot = base + b * kBlkK + tid;
      uint32_t o = 0;
      if (tid < kb) {
        o = outcome_bit(seed, circuit, shot0 + sh, m0 + slot);
        t.out[size_t(slot) * S + sh] = uint8_t(o);
        if (sh == 0) t.kind[slot] = 1;
      }
      const uint64_t ob = __ballot(o != 0);
      if (lane == 0) {
        s_rp = uint32_t(rp);
        s_o = uint32_t(ob);
      }
    }
    __syncthreads();
    const uint32_t rp = s_rp, ob = s_o;
#pragma unroll
    for (uint32_t j = 0; j < 2; ++j) {
      const uint32_t w = tid + j * kBlkSignThreads;
      if (w >= W) continue;
      uint64_t kill = 0, set = 0;
      for (uint32_t i = 0; i < kb; ++i) {
        const uint32_t p = s_P[i], pn = p - n;
        if ((p >> 6) == w) {
          kill |= bbit(p);
          if ((ob >> i) & 1u) set |= bbit(p);
        }
        if ((pn >> 6) == w) kill |= bbit(pn);
      }
      uint64_t v = (r[j] & ~kill) ^ h[j];
#pragma unroll
      for (uint32_t i = 0; i < kBlkK; ++i) v ^= ((rp >> i) & 1u) ? u[j][i] : 0ull;
      r[j] = v | set;
    }
    done += kb;
    __syncthreads();
  }
  (void)done;
#pragma unroll
  for (uint32_t j = 0; j < 2; ++j) {
    const uint32_t w = tid + j * kBlkSignThreads;
    if (w < W) t.R[size_t(w) * S + sh] = r[j];
  }
}

}  // namespace

// Launch shape of the blocked pass for n qubits: G sweeper workgroups (plus
// one planner) with L row words per lane and L columns per wave.
bool blk_shape(uint32_t n, uint32_t num_cus, uint32_t *G, uint32_t *L) {
  if (!persist_layout(n)) return false;
  const uint32_t W = (2 * n + 63) / 64;
  const uint32_t l = (W + 63) / 64;
  const uint32_t per = kBlkWaves * l;
  const uint32_t g = (n + per - 1) / per;
  if (g + 1 > num_cus || g + 1 > kPersistMaxGroups) return false;
  *G = g;
  *L = l;
  return true;
}

size_t blk_lds_bytes(uint32_t L) { return size_t(kBlkK) * 64 * L * 8; }

hipError_t launch_blk_chunk(const TabDev &t, const BlkDev &s, const uint32_t *dev_qubits, uint32_t cnt,
                            uint32_t G, uint32_t L, uint32_t abort_at, hipStream_t st) {
  if (cnt == 0 || cnt > kPersistMaxChunk || (cnt + kBlkK - 1) / kBlkK > s.NB || L < 1 || L > 5)
    return hipErrorInvalidValue;
  const void *fns[5] = {reinterpret_cast<const void *>(k_blk<1>), reinterpret_cast<const void *>(k_blk<2>),
                        reinterpret_cast<const void *>(k_blk<3>), reinterpret_cast<const void *>(k_blk<4>),
                        reinterpret_cast<const void *>(k_blk<5>)};
  static bool attr_set[5] = {false, false, false, false, false};
  if (!attr_set[L - 1]) {
    hipError_t e = hipFuncSetAttribute(fns[L - 1], hipFuncAttributeMaxDynamicSharedMemorySize,
                                       int(blk_lds_bytes(L)));
    if (e != hipSuccess) return e;
    attr_set[L - 1] = true;
  }
  k_blk_begin<<<1, 256, 0, st>>>(s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  BlkArgs a{dev_qubits, cnt, G, abort_at};
  TabDev targ = t;
  BlkDev sarg = s;
  void *args[] = {&targ, &sarg, &a};
  return hipLaunchCooperativeKernel(fns[L - 1], dim3(G + 1), dim3(kBlkThreads), args, blk_lds_bytes(L), st);
}

hipError_t launch_blk_finalize(const TabDev &t, const BlkDev &s, uint32_t cnt, uint32_t base, uint64_t seed,
                               uint64_t circuit, uint64_t shot0, uint64_t m0, uint32_t G, hipStream_t st) {
  const uint32_t nb = (cnt + kBlkK - 1) / kBlkK;
  k_blk_patch<<<nb, kBlkK, 0, st>>>(t, s);
  k_blk_reduce<<<dim3(nb, (t.W + 255) / 256), 256, 0, st>>>(t, s, G);
  k_blk_signs<<<t.S, kBlkSignThreads, 0, st>>>(t, s, cnt, base, seed, circuit, shot0, m0);
  return hipGetLastError();
}

}  // namespace cliff
