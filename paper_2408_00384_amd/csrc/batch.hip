// Batched circuits: one persistent launch runs thousands of independent small
// circuits, each held entirely in LDS by one workgroup ("team").
//
// Per circuit (phase-space method of the paper's Sec. 2, after Aaronson &
// Gottesman 2004): |0...0> tableau, every gate layer, then Z-measurement of
// every qubit in ascending order for all shots at once (x/z evolve once, the
// signs of each shot sit in their own bit column).  Rules are those of the
// HBM path: H/S/CNOT column updates; rowsum with the phase function g counted
// in bit-sliced mod-4 counters; smallest-pivot random branch with Philox
// outcomes keyed by (seed; measurement, shot, circuit); deterministic branch
// from the sign of the product of the selected stabilizers.
//
// Work distribution: workgroups pull circuit indices from a device counter in
// the order given by the host (largest first), until the list is exhausted.
// LDS per team, sized at launch for the largest circuit of the launch (maxn
// qubits, MW = ceil(2 maxn / 64) row words, MWl the power of two >= MW, SS =
// most shots): X[j][w] and Z[j][w] (column-major, column stride Wl = the power
// of two >= the circuit's W, maxn * MWl words each), signs R[w][s] (MW * SS),
// pending gate signs (MW), the waves' counter slots (two sets of 2 * waves *
// MWl), the next measured column's x words (two sets of MW) and the random
// outcome bits (maxn * SS bits).
// Occupancy follows from that size, so a launch of small circuits keeps more
// teams per compute unit.
//
// LDS banks (64 of 4 bytes): with the power-of-two column stride, column j
// starts at bank 2 Wl j mod 64, so a gate op's accesses fall in one of 32 / Wl
// bank ranges set by its qubit (mod 32 / Wl; for W >= 5, two half-ranges
// picked by the op's slot parity).  The ops of a layer commute, and
// cliff_batch_order_ops arranges them so the ops sharing a 32-lane access
// group use distinct ranges.
#include <algorithm>
#include <vector>

#include "internal.h"
#include "philox.h"

namespace cliff {

// Number of ops a gate-loop step applies per thread, as a type.
template <int N>
struct OpCount {
  static constexpr int value = N;
};

struct BatchDescDev {
  uint32_t n, depth, shots, reserved;
  uint64_t ops_off, offs_off, out_off, circuit_id;
};

// LDS words of a launch (the kernel carves its dynamic LDS the same way).
struct BatchLds {
  uint32_t mw, mwl, ss, words;
  __host__ __device__ BatchLds(uint32_t maxn, uint32_t max_shots, uint32_t nwave) {
    mw = (2 * maxn + 63) / 64;
    mwl = mw <= 1 ? 1u : (1u << (32 - __builtin_clz(mw - 1)));
    ss = max_shots;
    words = 2 * maxn * mwl + mw * ss + mw + 4 * nwave * mwl + 2 * mw + (maxn * ss + 63) / 64;
  }
};

template <int TEAM>
__global__ void __launch_bounds__(TEAM) k_batch(const BatchDescDev *__restrict__ descs,
                                               const uint64_t *__restrict__ ops,
                                               const uint32_t *__restrict__ offs,
                                               uint8_t *__restrict__ out,
                                               const uint32_t *__restrict__ order, uint32_t count,
                                               uint64_t seed, uint32_t *queue, uint32_t *errors,
                                               uint32_t maxn, uint32_t max_shots) {
  constexpr int NWAVE = TEAM / 64;
  extern __shared__ uint64_t s_dyn[];
  const BatchLds lay(maxn, max_shots, NWAVE);
  const uint32_t SS = lay.ss;                    // sign stride (shots)
  uint64_t *const sX = s_dyn;
  uint64_t *const sZ = sX + maxn * lay.mwl;
  uint64_t *const sR = sZ + maxn * lay.mwl;      // signs, stride SS
  uint64_t *const sP = sR + lay.mw * SS;         // gate sign flips (same for every shot)
  uint64_t *const sC0 = sP + lay.mw;             // counter slots, two sets (measurement parity)
  uint64_t *const sC1 = sC0 + 2 * NWAVE * lay.mwl;
  uint64_t *const sN = sC1 + 2 * NWAVE * lay.mwl; // column of the next measurement, two sets
  uint64_t *const sO = sN + 2 * lay.mw;           // random outcome bits, bit m * S + shot
  __shared__ uint32_t s_circ, s_par[2], s_y[2];
  const uint32_t tid = threadIdx.x, lane = tid & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);

  for (;;) {
    if (tid == 0) {
      const uint32_t q = atomicAdd(queue, 1u);
      s_circ = q < count ? order[q] : kNone;
    }
    __syncthreads();
    const uint32_t ci = s_circ;
    if (ci == kNone) return;
    const BatchDescDev d = descs[ci];
    const uint32_t n = d.n, S = d.shots;
    if (n == 0 || n > maxn || S == 0 || S > SS) {
      if (tid == 0) atomicAdd(errors, 1u);
      __syncthreads();
      continue;
    }
    const uint32_t W = (2 * n + 63) / 64;
    const uint32_t Wl = W <= 1 ? 1u : (1u << (32 - __builtin_clz(W - 1)));   // pow2 >= W: column stride
    // ---- |0...0> (the padding words past W are never read)
    for (uint32_t i = tid; i < n * Wl; i += TEAM) {
      const uint32_t j = i / Wl, w = i % Wl, zr = n + j;
      sX[i] = (w == (j >> 6)) ? (1ull << (j & 63)) : 0ull;
      sZ[i] = (w == (zr >> 6)) ? (1ull << (zr & 63)) : 0ull;
    }
    for (uint32_t i = tid; i < W * SS; i += TEAM) sR[i] = 0;
    // the Philox bit of every (measurement, shot), all waves at once, packed
    // 64 to a word by a ballot: the measurement loop then reads its bits
    // instead of running the generator on the sign-updating wave
    for (uint32_t base = wave * 64; base < n * S; base += TEAM) {
      const uint32_t i = base + lane;
      const uint32_t bit = i < n * S ? outcome_bit(seed, d.circuit_id, i % S, i / S) : 0u;
      const uint64_t word = __ballot(bit);
      if (lane == 0) sO[base / 64] = word;
    }
    if (tid < lay.mw) sP[tid] = 0;
    __syncthreads();
    // ---- gate layers: thread <-> (op, K row words).  From W = 5 on K = 2, the
    // two words as one 128-row value: the op's decode and its single-qubit
    // masks serve both and a layer needs half the passes; below that the
    // threads per op are few already and K = 1.  With K = 2 the four threads
    // of an op hold words t and t + 4 (t = 0..3), the first of the two
    // accesses reading word t in even op slots and word t + 4 in odd ones, so
    // the two halves of a column's banks serve two ops at once.  A thread's
    // words are fixed, so the sign flips it produces accumulate in registers
    // for the whole circuit.
    {
      const uint64_t *cops = ops + d.ops_off;
      const uint32_t *coffs = offs + d.offs_off;
      // The next layer's bounds and this thread's first two ops of it are
      // loaded one layer ahead, so a layer does not start with a chain of
      // dependent global loads (reads stay inside the circuit's ops).  Layers
      // and measurement steps meet at LDS-only barriers: they share nothing
      // else, and a full barrier would also wait for those prefetches and for
      // the outcome stores.
      const uint32_t depth = d.depth, end = coffs[depth];
      // every prefetch is an unconditional load from an in-bounds address (the
      // circuit's last op, or its descriptor when it has none) and the value is
      // selected after, so the compiler counts the loads in flight exactly
      const uint64_t *safe = end ? cops + (end - 1) : reinterpret_cast<const uint64_t *>(descs + ci);
      auto fetch = [&](uint32_t k) -> uint64_t {
        const uint64_t v = *(k < end ? cops + k : safe);
        return k < end ? v : 0ull;
      };
      auto gates = [&](auto zero) {
        using T = decltype(zero);
        constexpr uint32_t K = sizeof(T) / 8;
        const uint32_t Wt = (W + K - 1) / K;                                        // threads per op
        const uint32_t Wq = Wt <= 1 ? 1u : (1u << (32 - __builtin_clz(Wt - 1)));   // pow2 >= Wt
        const uint32_t t = tid % Wq, k0 = tid / Wq, kst = TEAM / Wq;
        // Words past W up to the column stride Wl are padding: the threads
        // holding them load, update and store them like the others (no
        // branches), and nothing else reads them.  K = 2: Wq = 4, W in 5..8,
        // Wl = 8.
        const uint32_t w0 = K == 2 ? t + 4 * (k0 & 1u) : t, w1 = t + 4 * ((k0 & 1u) ^ 1u);
        const bool hl = w0 < W, hh = K == 2 && w1 < W;
        const uint32_t stride = K == 2 ? 8u : Wl;   // column stride (words); 8 whenever K = 2
        // this thread's words of column 0 in X and Z; column c is c * stride
        // words on
        uint64_t *const xl = sX + w0, *const zl = sZ + w0, *const xh = sX + w1, *const zh = sZ + w1;
        T racc = zero;
        auto load = [&](uint64_t *lo, uint64_t *hi, uint32_t c) -> T {
          if constexpr (K == 2) return T{lo[c * stride], hi[c * stride]};
          else return lo[c * stride];
        };
        auto store = [&](uint64_t *lo, uint64_t *hi, uint32_t c, T v) {
          if constexpr (K == 2) {
            lo[c * stride] = v.lo;
            hi[c * stride] = v.hi;
          } else {
            lo[c * stride] = v;
          }
        };
        // Two ops on this thread's row words (ops of a layer act on distinct
        // qubits, so their columns are distinct): all loads of both first, so
        // the second op's reads do not wait behind the first op's writes.
        // Loads are unconditional (an absent or malformed op reads column 0, a
        // single-qubit op its own column twice); stores only for present ops.
        auto apply = [&](auto count, uint64_t op0, bool has_op0, uint64_t op1, bool has_op1) {
          constexpr int N = decltype(count)::value;   // 1 when no lane of the wave has a second op
          uint32_t a[2], b[2], pr[2], ca[2], cb[2];
          bool go[2];
#pragma unroll
          for (int u = 0; u < N; ++u) {
            const uint64_t op = u ? op1 : op0;
            const bool has = u ? has_op1 : has_op0;
            go[u] = has && op_valid(op, n);
            if (has && !go[u]) atomicAdd(errors, 1u);   // malformed op
            a[u] = go[u] ? op_a(op) : 0u;
            pr[u] = go[u] ? op_pair(op) : uint32_t(PAIR_NONE);
            b[u] = pr[u] != PAIR_NONE ? op_b(op) : a[u];
            ca[u] = go[u] ? op_ca(op) : 0u;
            cb[u] = pr[u] != PAIR_NONE ? op_cb(op) : 0u;
          }
          T xa[2], za[2], xb[2], zb[2];
#pragma unroll
          for (int u = 0; u < N; ++u) {
            xa[u] = load(xl, xh, a[u]);
            za[u] = load(zl, zh, a[u]);
            xb[u] = load(xl, xh, b[u]);
            zb[u] = load(zl, zh, b[u]);
          }
          // code 0 is the identity, so the single-qubit updates run without a
          // branch (nearly every op has one).  When the wave's two-qubit ops
          // are all CNOTs (a wave-uniform test), the CNOT runs under a lane
          // mask instead of the per-kind branches.
          bool other = false;
#pragma unroll
          for (int u = 0; u < N; ++u) other |= pr[u] != PAIR_NONE && pr[u] != PAIR_CNOT;
          const bool only_cnot = __ballot(other) == 0;
#pragma unroll
          for (int u = 0; u < N; ++u) {
            sq_apply(ca[u], xa[u], za[u], racc);
            sq_apply(cb[u], xb[u], zb[u], racc);   // cb = 0 without a second qubit
            if (only_cnot) {
              const T mc = mask_if<T>(pr[u] == PAIR_CNOT);
              racc ^= bop3<LUT_AND3>(mc, xa[u], bop3<LUT_AND_ANDN>(zb[u], mc, xb[u] ^ za[u]));
              xb[u] ^= xa[u] & mc;
              za[u] ^= zb[u] & mc;
            } else if (pr[u] != PAIR_NONE) {
              pair_apply(pr[u], xa[u], za[u], xb[u], zb[u], racc);
            }
          }
#pragma unroll
          for (int u = 0; u < N; ++u) {
            if (pr[u] != PAIR_NONE) {
              store(xl, xh, b[u], xb[u]);
              store(zl, zh, b[u], zb[u]);
            }
            if (go[u]) {
              store(xl, xh, a[u], xa[u]);
              store(zl, zh, a[u], za[u]);
            }
          }
        };
        uint32_t a0 = coffs[0], a1 = depth ? coffs[1] : a0;
        uint64_t f0 = fetch(a0 + k0), f1 = fetch(a0 + k0 + kst);
        for (uint32_t l = 0; l < depth; ++l) {
          const uint32_t b0 = a1, b1 = l + 2 <= depth ? coffs[l + 2] : a1;
          const uint64_t g0 = fetch(b0 + k0), g1 = fetch(b0 + k0 + kst);
          {
            // the two prefetched ops in straight-line code, so their wait does
            // not cover the loads just issued for the next layer; a wave none
            // of whose lanes has a second op applies one (wave-uniform test)
            if (a0 + k0 < a1) {
              const bool second = a0 + k0 + kst < a1;
              if (__ballot(second)) apply(OpCount<2>{}, f0, true, f1, second);
              else apply(OpCount<1>{}, f0, true, f1, false);
            }
            for (uint32_t k = a0 + k0 + 2 * kst; k < a1; k += 2 * kst) {
              const bool two = k + kst < a1;
              if (__ballot(two)) apply(OpCount<2>{}, cops[k], true, cops[two ? k + kst : k], two);
              else apply(OpCount<1>{}, cops[k], true, 0ull, false);
            }
          }
          lds_barrier();
          a0 = b0;
          a1 = b1;
          f0 = g0;
          f1 = g1;
        }
        auto flush = [&](uint32_t w, uint64_t v) {
          if (v) atomicXor(reinterpret_cast<unsigned long long *>(&sP[w]), (unsigned long long)v);
        };
        if constexpr (K == 2) {
          if (hl) flush(w0, racc.lo);
          if (hh) flush(w1, racc.hi);
        } else {
          if (hl) flush(w0, racc);
        }
      };
      if (W >= 5) gates(U128{0, 0});
      else gates(uint64_t(0));
      __syncthreads();
      for (uint32_t i = tid; i < W * SS; i += TEAM) sR[i] ^= sP[i / SS];
      __syncthreads();
    }
    // ---- measure every qubit
    const uint32_t cpw = 64 / Wl;                  // columns per wave instruction
    const uint32_t sub = lane / Wl, wl = lane % Wl;
    const uint32_t slots = NWAVE * cpw;            // column slots per pass
    const uint32_t slot = wave * cpw + sub;
    uint8_t *cout = out + d.out_off;
    // Pivot of measurement a (smallest stabilizer row with x_a = 1) and, per
    // lane word, its update mask (random) or product-row mask T
    // (deterministic); every wave computes them from the x words of column a
    // as staged in sN[a & 1] (the column itself may already be changing under
    // a wave that has gone on to sweep measurement a).
    auto select = [&](uint32_t a, uint32_t &p, uint64_t &m) {
      const uint64_t *col = sN + (a & 1u) * lay.mw;
      uint32_t cand = kNone;
      if (lane < W && lane >= (n >> 6)) {
        uint64_t v = col[lane];
        if (lane == (n >> 6)) v &= ~0ull << (n & 63);
        if (v) cand = lane * 64 + uint32_t(__builtin_ctzll(v));
      }
      // lane w holds word w, so the first lane with a candidate has the smallest row
      const uint64_t bal = __ballot(cand != kNone);
      p = bal ? uint32_t(__builtin_amdgcn_readlane(int(cand), int(__builtin_ctzll(bal)))) : kNone;
      m = 0;
      if (wl < W) {
        if (p != kNone) {
          m = col[wl];
          if (wl == (p >> 6)) m &= ~(1ull << (p & 63));
        } else {
          const uint32_t q = n >> 6, sh = n & 63;
          auto src = [&](int32_t i) -> uint64_t {
            if (i < 0 || i >= int32_t((n + 63) / 64)) return 0ull;
            uint64_t v = col[i];
            if (uint32_t(i) == q && sh) v &= (1ull << sh) - 1;
            return v;
          };
          const int32_t i = int32_t(wl) - int32_t(q);
          m = src(i) << sh;
          if (sh) m |= src(i - 1) >> (64 - sh);
        }
      }
    };
    // One barrier per measurement a, after the sweep (or the deterministic
    // sums): then every wave selects a + 1 from the staged column while wave
    // 0 sums the counters and updates the signs of a, and each wave goes on
    // to sweep a + 1 without waiting for wave 0.  That is safe because the
    // signs, the outcome bytes and the anomaly count are wave 0's alone; the
    // counter slots, the deterministic sums and the staged column are double
    // buffered by measurement parity (a set is written again two measurements
    // later, after a barrier that wave 0 reaches only once it has read it);
    // a column's words are read and written by one lane in program order
    // within the sweeps; and the deterministic branch, which reads every
    // column, does so before the barrier that any later sweep comes after.
    uint32_t p;
    uint64_t m;
    if (tid < W) sN[tid] = sX[tid];   // column 0 staged
    if (tid < 2) { s_par[tid] = 0; s_y[tid] = 0; }
    lds_barrier();
    select(0, p, m);
    const uint32_t own = slot;        // lanes (sub, wl) of this slot own columns j = slot (mod slots)
    for (uint32_t a = 0; a < n; ++a) {
      const uint32_t ab = a & 1u;
      uint64_t *const c0s = sC0 + ab * NWAVE * Wl, *const c1s = sC1 + ab * NWAVE * Wl;
      uint32_t p_next = kNone;
      uint64_t m_next = 0;
      if (p != kNone) {
        const uint32_t pn = p - n, wpn = pn >> 6, wp = p >> 6;
        const uint64_t bpn = 1ull << (pn & 63), bpb = 1ull << (p & 63);
        // this lane's bits of rows p - n and p (zero where its word holds
        // neither): overwritten in every column by the pivot row's bits, and
        // by x = 0, z = [column is a], as masked selects
        const uint64_t Bpn = wl == wpn ? bpn : 0ull, Bp = wl == wp ? bpb : 0ull, F = Bpn | Bp;
        uint64_t c0 = 0, c1 = 0;
        if (wl < W) {
          // two columns per pass, all loads first (distinct columns: the
          // second's reads need not wait for the first's writes)
          for (uint32_t j0 = slot; j0 < n; j0 += 2 * slots) {
            const uint32_t j1 = j0 + slots < n ? j0 + slots : j0;
            const bool two = j0 + slots < n;
            uint64_t xp[2], zp[2], xv[2], zv[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
              const uint32_t j = u ? j1 : j0;
              xp[u] = sX[j * Wl + wp];
              zp[u] = sZ[j * Wl + wp];
              xv[u] = sX[j * Wl + wl];
              zv[u] = sZ[j * Wl + wl];
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
              const uint32_t j = u ? j1 : j0;
              if (u && !two) break;
              const uint32_t xpj = uint32_t(xp[u] >> (p & 63)) & 1u;
              const uint32_t zpj = uint32_t(zp[u] >> (p & 63)) & 1u;
              const uint64_t x = xv[u], z = zv[u];
              const uint64_t X1 = mask_if<uint64_t>(xpj), Z1 = mask_if<uint64_t>(zpj);
              // rows in M anticommuting with the pivot's Pauli on column j (X:
              // z, Z: x, Y: x ^ z); g = +1 on them where (X: x; Z: ~z; Y: z),
              // else -1, and adding +-1 to the 2-bit counter flips c1 where c0
              // equals that condition: c1 ^= anti & ~(c0 ^ sel), c0 ^= anti
              const uint64_t anti = bop3<LUT_AND_XOR>(Z1, x, X1 & z) & m;
              const uint64_t sel = (Z1 & ~(z ^ X1)) | (~Z1 & x);
              c1 ^= bop3<LUT_AND_XNOR>(anti, c0, sel);
              c0 ^= anti;
              uint64_t nx = bop3<LUT_AND_XOR>(X1, m, x), nz = bop3<LUT_AND_XOR>(Z1, m, z);
              nx = (nx & ~F) | (X1 & Bpn);
              nz = (nz & ~F) | (Z1 & Bpn) | (mask_if<uint64_t>(j == a) & Bp);
              sX[j * Wl + wl] = nx;
              sZ[j * Wl + wl] = nz;
            }
          }
        }
        // counters: the cpw column slots of a word sit in lanes sub * Wl + wl
        // of one wave (same wl): mod-4 sums by a butterfly over them, then
        // the waves' sums through LDS
        for (uint32_t off = Wl; off < 64; off <<= 1) {
          const uint64_t b0 = __shfl_xor(c0, int(off)), b1 = __shfl_xor(c1, int(off));
          c1 ^= b1 ^ (c0 & b0);
          c0 ^= b0;
        }
        if (lane < Wl) {
          c0s[wave * Wl + lane] = c0;
          c1s[wave * Wl + lane] = c1;
        }
        // the owner lanes stage column a + 1 as measurement a left it
        if (a + 1 < n && wl < W && (a + 1) % slots == own)
          sN[(ab ^ 1u) * lay.mw + wl] = sX[(a + 1) * Wl + wl];
        lds_barrier();
        if (a + 1 < n) select(a + 1, p_next, m_next);
        // reduce counters per word (wave 0), then update the signs of all shots
        if (wave == 0) {
          // pivot signs of every shot (bit s = r_p of shot s)
          const uint32_t rb = lane < S ? uint32_t(sR[wp * SS + lane] >> (p & 63)) & 1u : 0u;
          const uint64_t rpw = __ballot(rb);
          uint64_t t0 = 0, t1 = 0;
          if (lane < Wl && lane < W) {
#pragma unroll
            for (int wv = 0; wv < NWAVE; ++wv) {
              const uint64_t b0 = c0s[wv * Wl + lane], b1 = c1s[wv * Wl + lane];
              t1 ^= b1 ^ (t0 & b0);
              t0 ^= b0;
            }
          }
          // one lane per (word, shot) pair; word values via shuffles (lane w
          // holds word w)
          for (uint32_t i0 = 0; i0 < W * S; i0 += 64) {
            const uint32_t i = i0 + lane, w = i / S, sh = i % S;
            const int src = int(i < W * S ? w : 0u);
            const uint64_t mw = __shfl(m, src);
            const uint64_t c1w = __shfl(t1, src);
            if (i < W * S) {
              const uint32_t rpb = uint32_t(rpw >> sh) & 1u;
              uint64_t rv = sR[w * SS + sh];
              rv ^= mw & (c1w ^ (rpb ? ~0ull : 0ull));
              if (w == wpn) rv = rpb ? (rv | bpn) : (rv & ~bpn);
              if (w == wp) {
                const uint32_t o = uint32_t(sO[(a * S + sh) / 64] >> ((a * S + sh) & 63)) & 1u;
                rv = o ? (rv | bpb) : (rv & ~bpb);
                cout[size_t(sh) * n + a] = uint8_t(o);
              }
              sR[w * SS + sh] = rv;
            }
          }
          const uint64_t bad = (lane < W) ? (t0 & m & ~(lane == wpn ? bpn : 0ull)) : 0ull;
          if (bad) atomicAdd(errors + 1, 1u);
        }
      } else {
        // deterministic: per column, pairs s < t in T with z_s x_t, and Y count
        uint32_t par = 0, ycnt = 0;
        for (uint32_t j = tid; j < n; j += TEAM) {
          uint32_t carry = 0;
          for (uint32_t w = 0; w < W; ++w) {
            // T mask of word w: lane w of every wave holds it
            const uint32_t q = n >> 6, sh = n & 63;
            uint64_t Tw = 0;
            {
              const int32_t i = int32_t(w) - int32_t(q);
              auto src = [&](int32_t ii) -> uint64_t {
                if (ii < 0 || ii >= int32_t((n + 63) / 64)) return 0ull;
                uint64_t v = sX[a * Wl + ii];
                if (uint32_t(ii) == q && sh) v &= (1ull << sh) - 1;
                return v;
              };
              Tw = src(i) << sh;
              if (sh) Tw |= src(i - 1) >> (64 - sh);
            }
            const uint64_t xt = sX[j * Wl + w] & Tw, zt = sZ[j * Wl + w] & Tw;
            ycnt += uint32_t(__popcll(xt & zt));
            uint64_t pre = zt << 1;
            pre ^= pre << 1; pre ^= pre << 2; pre ^= pre << 4;
            pre ^= pre << 8; pre ^= pre << 16; pre ^= pre << 32;
            par ^= (uint32_t(__popcll(xt & pre)) & 1u) ^ (carry & uint32_t(__popcll(xt)) & 1u);
            carry ^= uint32_t(__popcll(zt)) & 1u;
          }
        }
        if (par & 1u) atomicXor(&s_par[ab], 1u);
        if (ycnt) atomicAdd(&s_y[ab], ycnt);
        // measurement a changed nothing: column a + 1 staged as it stands
        if (a + 1 < n && wl < W && (a + 1) % slots == own)
          sN[(ab ^ 1u) * lay.mw + wl] = sX[(a + 1) * Wl + wl];
        lds_barrier();
        if (a + 1 < n) select(a + 1, p_next, m_next);
        if (wave == 0) {
          // shuffles with the whole wave active (lane w holds mask word w)
          uint32_t rt = 0;
          for (uint32_t w = 0; w < W; ++w) {
            const uint64_t Tw = __shfl(m, int(w));
            if (lane < S) rt ^= uint32_t(__popcll(Tw & sR[w * SS + lane])) & 1u;
          }
          const uint32_t par_a = s_par[ab], y_a = s_y[ab];
          if (lane < S) cout[size_t(lane) * n + a] = uint8_t(rt ^ (par_a & 1u) ^ ((y_a >> 1) & 1u));
          if (lane == 0 && (y_a & 1u)) atomicAdd(errors + 1, 1u);
          if (lane == 0) { s_par[ab] = 0; s_y[ab] = 0; }   // after wave 0's reads above
        }
      }
      p = p_next;
      m = m_next;
    }
  }
}

// ---- host: op order within a layer for the batch kernel's LDS banks -------
//
// For a circuit with W row words, the kernel's 32-lane access groups hold P
// consecutive ops of a layer (P = 32 / Wq, Wq = threads per op), and an op's
// column accesses fall in bank range (qubit mod P): P = 8, 16, 32 for W = 3..4,
// 2, 1.  For W >= 5 a group holds 8 ops, its even and odd slots using the two
// halves of a column's banks, so each half needs distinct (qubit mod 4).  A
// group (half) is free of bank conflicts when its ops' first qubits are in
// distinct classes, and so are their second qubits (a single-qubit op's
// second access reads its own column again): a bipartite matching between
// first-qubit and second-qubit classes.  Each group takes a
// maximum matching, found by augmenting paths that try the class pairs with
// the most ops left first (which keeps the classes balanced for the groups
// after it); its free slots take ops from the fullest class pairs.
namespace {

struct LayerOrder {
  static constexpr uint32_t kMaxP = 32;
  uint32_t P = 0, nb = 0;
  // ops grouped by class pair (a, b), key a * (P + 1) + b: pool[head[k] .. tail[k])
  std::vector<uint64_t> pool;
  std::vector<uint32_t> head, tail;
  uint32_t leftA[kMaxP];
  int matchA[kMaxP], matchB[kMaxP];
  char seen[kMaxP];

  uint32_t size(uint32_t ca, uint32_t cb) const {
    const uint32_t k = ca * (P + 1) + cb;
    return tail[k] - head[k];
  }
  uint64_t pop(uint32_t k) {
    leftA[k / (P + 1)]--;
    return pool[--tail[k]];
  }

  // augmenting path from first-qubit class ca (second classes with the most
  // ops left tried first); matchA[ca] = its second class
  bool augment(uint32_t ca) {
    uint32_t cand[kMaxP + 1], nc = 0;
    for (uint32_t cb = 0; cb <= P; ++cb)
      if (size(ca, cb)) {
        uint32_t at = nc++;   // insertion by size, most first (stable)
        while (at > 0 && size(ca, cand[at - 1]) < size(ca, cb)) {
          cand[at] = cand[at - 1];
          --at;
        }
        cand[at] = cb;
      }
    for (uint32_t k = 0; k < nc; ++k) {
      const uint32_t cb = cand[k];
      if (cb == P) {
        matchA[ca] = int(P);
        return true;
      }
      if (seen[cb]) continue;
      seen[cb] = 1;
      if (matchB[cb] < 0 || augment(uint32_t(matchB[cb]))) {
        matchA[ca] = int(cb);
        matchB[cb] = int(ca);
        return true;
      }
    }
    return false;
  }

  // up to `slots` ops for one conflict-free group (half), appended to out
  void take_group(uint32_t slots, std::vector<uint64_t> &out) {
    uint32_t order[kMaxP];
    for (uint32_t ca = 0; ca < P; ++ca) {   // first-qubit classes with the most ops left first
      matchA[ca] = matchB[ca] = -1;
      uint32_t at = ca;
      while (at > 0 && leftA[order[at - 1]] < leftA[ca]) {
        order[at] = order[at - 1];
        --at;
      }
      order[at] = ca;
    }
    uint32_t got = 0;
    for (uint32_t r = 0; r < P && got < slots; ++r) {
      const uint32_t ca = order[r];
      if (!leftA[ca]) break;
      for (uint32_t k = 0; k < P; ++k) seen[k] = 0;
      if (augment(ca)) ++got;
    }
    for (uint32_t ca = 0; ca < P; ++ca)
      if (matchA[ca] >= 0) out.push_back(pop(ca * (P + 1) + uint32_t(matchA[ca])));
    for (; got < slots; ++got) {   // no conflict-free op left: the fullest class pair
      uint32_t best = 0, bi = nb;
      for (uint32_t k = 0; k < nb; ++k)
        if (tail[k] - head[k] > best) {
          best = tail[k] - head[k];
          bi = k;
        }
      if (bi == nb) break;
      out.push_back(pop(bi));
    }
  }

  void run(uint64_t *ops, uint32_t cnt, uint32_t W, std::vector<uint64_t> &tmp) {
    if (cnt <= 1) return;
    const bool halves = W >= 5;
    if (halves) {
      P = 4;
    } else {
      const uint32_t wq = W <= 1 ? 1u : (1u << (32 - __builtin_clz(W - 1)));
      P = 32 / wq;
    }
    nb = P * (P + 1);
    // the kernel's second access of a single-qubit op reads its own column again
    auto key = [&](uint64_t op) {
      return (op_a(op) % P) * (P + 1) + (op_pair(op) != PAIR_NONE ? op_b(op) : op_a(op)) % P;
    };
    head.assign(nb + 1, 0);
    for (uint32_t k = 0; k < cnt; ++k) head[key(ops[k]) + 1]++;
    for (uint32_t k = 0; k < nb; ++k) head[k + 1] += head[k];
    tail.assign(head.begin(), head.end() - 1);
    pool.resize(cnt);
    for (uint32_t k = cnt; k-- > 0;) pool[tail[key(ops[k])]++] = ops[k];   // reversed: pops give stream order
    for (uint32_t ca = 0; ca < P; ++ca) leftA[ca] = head[(ca + 1) * (P + 1)] - head[ca * (P + 1)];
    tmp.clear();
    while (tmp.size() < cnt) {
      const uint32_t rest = cnt - uint32_t(tmp.size());
      if (!halves) {
        take_group(std::min(P, rest), tmp);
      } else {
        uint64_t ev[8], od[8];
        std::vector<uint64_t> &buf = tmp;   // the two halves, interleaved slot by slot
        const size_t at = buf.size();
        take_group(std::min(4u, (rest + 1) / 2), buf);
        const uint32_t ne = uint32_t(buf.size() - at);
        for (uint32_t k = 0; k < ne; ++k) ev[k] = buf[at + k];
        buf.resize(at);
        take_group(std::min(4u, rest - ne), buf);
        const uint32_t no = uint32_t(buf.size() - at);
        for (uint32_t k = 0; k < no; ++k) od[k] = buf[at + k];
        buf.resize(at);
        for (uint32_t k = 0; k < 4; ++k) {
          if (k < ne) buf.push_back(ev[k]);
          if (k < no) buf.push_back(od[k]);
        }
      }
    }
    std::copy(tmp.begin(), tmp.end(), ops);
  }
};

}  // namespace

int batch_order_ops(uint32_t n, uint64_t *ops, const uint32_t *offs, uint32_t depth) {
  if (n < 1 || n > kBatchMaxN || !offs) return -1;
  for (uint32_t l = 0; l < depth; ++l)
    if (offs[l + 1] < offs[l]) return -1;
  if (offs[depth] > offs[0] && !ops) return -1;
  const uint32_t W = (2 * n + 63) / 64;
  std::vector<uint64_t> tmp;
  LayerOrder lo;
  for (uint32_t l = 0; l < depth; ++l) lo.run(ops + offs[l], offs[l + 1] - offs[l], W, tmp);
  return 0;
}

// Teams per compute unit for a launch's LDS size.
template <int TEAM>
static uint32_t batch_grid(size_t lds_bytes, int num_cus) {
  int per = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_batch<TEAM>, TEAM, lds_bytes) != hipSuccess ||
      per < 1)
    per = 1;
  return uint32_t(per) * uint32_t(num_cus);
}

template <int TEAM>
static hipError_t launch_batch_t(const BatchDescDev *descs, const uint64_t *ops, const uint32_t *offs,
                                 uint8_t *out, const uint32_t *order, uint32_t count, uint64_t seed,
                                 uint32_t *queue, uint32_t *errors, uint32_t maxn, uint32_t max_shots,
                                 int num_cus, hipStream_t st) {
  const size_t lds = size_t(BatchLds(maxn, max_shots, TEAM / 64).words) * 8;
  k_batch<TEAM><<<batch_grid<TEAM>(lds, num_cus), TEAM, lds, st>>>(descs, ops, offs, out, order, count, seed,
                                                                   queue, errors, maxn, max_shots);
  return hipGetLastError();
}

// work[0] = queue head, work[1] = rejected descriptors, work[2] = anomalies
__global__ void k_reset_queue(uint32_t *work) {
  if (threadIdx.x < 4) work[threadIdx.x] = 0;
}

hipError_t launch_batch(const void *descs, const uint64_t *ops, const uint32_t *offs, uint8_t *out,
                        const uint32_t *order, uint32_t count, uint64_t seed, uint32_t *work,
                        uint32_t team, uint32_t maxn, uint32_t max_shots, int num_cus, hipStream_t st) {
  if (maxn < 1 || maxn > kBatchMaxN || max_shots < 1 || max_shots > 64) return hipErrorInvalidValue;
  if (team != 64 && team != 128 && team != 256 && team != 512 && team != 1024) return hipErrorInvalidValue;
  const BatchDescDev *d = reinterpret_cast<const BatchDescDev *>(descs);
  k_reset_queue<<<1, 64, 0, st>>>(work);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  uint32_t *q = work, *err = work + 1;
  switch (team) {
    case 64: return launch_batch_t<64>(d, ops, offs, out, order, count, seed, q, err, maxn, max_shots, num_cus, st);
    case 128: return launch_batch_t<128>(d, ops, offs, out, order, count, seed, q, err, maxn, max_shots, num_cus, st);
    case 256: return launch_batch_t<256>(d, ops, offs, out, order, count, seed, q, err, maxn, max_shots, num_cus, st);
    case 512: return launch_batch_t<512>(d, ops, offs, out, order, count, seed, q, err, maxn, max_shots, num_cus, st);
    default: return launch_batch_t<1024>(d, ops, offs, out, order, count, seed, q, err, maxn, max_shots, num_cus, st);
  }
}

}  // namespace cliff
