// Measuring a list of qubits with the tableau held in registers and LDS,
// in chunks of up to Kc measurements; per chunk four launches: publish the
// first measured column, the cooperative x/z kernel, a parallel reduction of
// the sign counters, and a per-shot sign walk.
//
// The method is that of measure_step.hip (paper Sec. 2, after Aaronson &
// Gottesman 2004: smallest-pivot random branch with rowsum and the phase
// function g counted in bit-sliced mod-4 counters; deterministic branch from
// the sign of the product of the selected stabilizers).  Only where the data
// lives and how workgroups meet differs:
//
//  * x/z kernel (k_meas_xz): G workgroups of 8 waves (two per SIMD).
//    Workgroup g owns the columns j = g (mod G), so consecutive qubits belong
//    to different workgroups, and wave v of it the workgroup's columns
//    c = v (mod 8).  A wave holds CW = L whole columns: lane l has row
//    words l, l + 64, ... (L = ceil(W / 64) <= 5 of them) of each, x bits in
//    registers and z bits in LDS, for the whole chunk, so the rowsum sweep
//    touches no HBM and the per-column decisions (the pivot row's Pauli on
//    the column) are taken once per column rather than once per 64 rows.
//    Between workgroups only measured columns travel: right after its sweep
//    of measurement m, the owner of a_{m+2} publishes that column as it
//    stands after measurement m, as tagged 64-bit entries (32 data bits and
//    the 32-bit slot tag in one atomic store, so a reader knows each entry is
//    complete without a separate flag or fence).  Every workgroup issues the
//    loads of that column (its words spread over the threads, plus the pivot
//    row's word) at the start of iteration m + 1 and uses them after its
//    sweep: each thread applies measurement m + 1's update to its words
//    (x ^= M where the pivot row has x = 1 on that column; rows p-n and p
//    rewritten) and the workgroup takes the smallest stabilizer row with
//    x = 1 as the next pivot.  The cross-workgroup latency is hidden behind a
//    whole sweep; each iteration costs three LDS-only barriers.  The waves'
//    mod-4 counters are summed in LDS with atomic XORs (the XOR's old value
//    gives the carry into the high plane) and each workgroup writes its
//    (c0, c1) pair per row word for every measurement of the chunk to HBM.
//  * reduce kernel: c1[m][w] = mod-4 sum of the partials of all workgroups.
//  * sign kernel: one workgroup per shot walks the chunk in order with that
//    shot's sign column in registers: r ^= M & (c1 ^ r_p), rows p-n and p
//    rewritten, outcome = Philox bit; deterministic outcomes from the XOR of
//    the product rows' signs and the two x/z terms accumulated by the x/z
//    kernel.  It runs on a second stream beside the next chunk's x/z kernel.
//
// Every wait is bounded; a timeout raises a device-wide abort flag that every
// wait checks, so all waves leave the kernel and the host reports the error.
#include "internal.h"
#include "philox.h"

namespace cliff {

constexpr uint32_t kSpinLimit = 1u << 20;   // polling rounds before giving up (~seconds)
constexpr uint32_t kWaves = 8;              // waves of an x/z workgroup (two per SIMD, 256 VGPRs each)
constexpr uint32_t kThreads = kWaves * 64;
constexpr uint32_t kWordsPerThread = (kPersistMaxWp + kThreads - 1) / kThreads;   // row words t, t + 512, ...

struct PersistArgs {
  const uint32_t *qubits;   // device, this chunk's k entries
  uint32_t k, G;
  uint32_t abort_at;        // measurement of this chunk at which every workgroup stops as if
                            // a wait had timed out (kNone: never; a test aid for the error path)
  const uint32_t *skip;     // device: leading measurements of the chunk already done by the
                            // blocked pass (null: none)
};

// The chunk's measurements left after the blocked pass (its count of done
// measurements in device memory, written by the kernel before this one).
__device__ __forceinline__ uint32_t chunk_skip(const uint32_t *skip) { return skip ? *skip : 0u; }

__device__ __forceinline__ uint64_t pbit(uint32_t b) { return 1ull << (b & 63); }

__device__ __forceinline__ uint32_t ld_relaxed(const uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_relaxed64(const uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed64(uint64_t *p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}


// Destabilizer half of a column shifted up by n rows (word w).
__device__ __forceinline__ uint64_t det_word(const uint64_t *col, uint32_t n, uint32_t NW, uint32_t W,
                                             uint32_t w) {
  if (w >= W) return 0ull;
  const uint32_t q = n >> 6, sh = n & 63;
  auto src = [&](int64_t i) -> uint64_t {
    if (i < 0 || i >= int64_t(NW)) return 0ull;
    uint64_t v = col[i];
    if (uint32_t(i) == q && sh) v &= pbit(sh) - 1;
    return v;
  };
  const int64_t i = int64_t(w) - int64_t(q);
  uint64_t v = src(i) << sh;
  if (sh) v |= src(i - 1) >> (64 - sh);
  return v;
}

// Entry pair of word w of published slot j; the data when both carry the
// slot's tag.
__device__ __forceinline__ bool tagged_word(uint64_t lo, uint64_t hi, uint32_t j, uint64_t *out) {
  const uint64_t tag = uint64_t(j + 1) << 32, hi_mask = ~0xffffffffull;
  *out = (lo & 0xffffffffull) | (hi << 32);
  return (lo & hi_mask) == tag && (hi & hi_mask) == tag;
}

// Wait for word w of published slot j (pub: the slots, Wp: their stride in
// words); false when the wait gave up or another workgroup raised the abort
// flag.
__device__ __forceinline__ bool wait_published(const uint64_t *pub, uint32_t Wp, uint32_t *abort_flag,
                                               uint32_t j, uint32_t w, uint64_t *out) {
  const uint64_t *src = pub + size_t(j) * 2 * Wp + 2 * w;
  uint32_t spins = 0;
  while (!tagged_word(ld_relaxed64(src), ld_relaxed64(src + 1), j, out)) {
    if (ld_relaxed(abort_flag)) return false;
    if (++spins > kSpinLimit) {
      atomicOr(abort_flag, 1u);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  return true;
}

// Smallest stabilizer row with x = 1 in word w (value v) of a column, or kNone.
__device__ __forceinline__ uint32_t pivot_candidate(uint64_t v, uint32_t w, uint32_t n, uint32_t W) {
  if (w >= W || w < (n >> 6)) return kNone;
  if (w == (n >> 6)) v &= ~0ull << (n & 63);
  return v ? w * 64 + uint32_t(__builtin_ctzll(v)) : kNone;
}

// Minimum of a wave's candidates when lane l holds word 64 * wave + l (the
// first lane with a candidate has the smallest); lane 0 folds it into *dst.
__device__ __forceinline__ void wave_min_into(uint32_t cand, uint32_t lane, uint32_t *dst) {
  const uint64_t bal = __ballot(cand != kNone);
  if (bal) {
    const uint32_t l = uint32_t(__builtin_ctzll(bal));
    const uint32_t v = uint32_t(__builtin_amdgcn_readlane(int(cand), int(l)));
    if (lane == 0) atomicMin(dst, v);
  }
}

template <int L, int CW>
__global__ void __launch_bounds__(kThreads) k_meas_xz(TabDev t, PersistArgs a) {
  // x bits of the owned columns live in registers, z bits in LDS:
  // z of slot k, word i of this lane at sZ[((wave * CW + k) * L + i) * 64 + lane]
  __shared__ uint64_t sZ[kWaves * CW * L * 64];
  __shared__ uint64_t s_col[2][kPersistMaxWp];          // column of measurement m in s_col[m & 1]
  __shared__ unsigned long long s_s0[kPersistMaxWp], s_s1[kPersistMaxWp];   // workgroup counter sums
  __shared__ uint32_t s_q[kPersistMaxChunk];            // this chunk's measured qubits
  __shared__ uint32_t s_p[2];                           // pivot row of measurement m in s_p[m & 1]
  __shared__ uint32_t s_abort, s_par, s_y;
  const uint32_t tid = threadIdx.x, lane = tid & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const uint32_t g = blockIdx.x, G = a.G;
  const uint32_t n = t.n, W = t.W;
  const uint32_t C = g < n ? (n - g + G - 1) / G : 0;   // owned columns g, g+G, g+2G, ...
  // slots k < ns of this wave hold columns c = wave + 8 k < C (wave-uniform)
  const uint32_t ns = C > wave ? (C - wave + kWaves - 1) / kWaves : 0;
  // thread t carries row words t + kThreads j (j < kWordsPerThread) of the measured columns
  uint64_t *zw = sZ + size_t(wave) * CW * L * 64 + lane;   // z of slot k, word i at zw[(k * L + i) * 64]

  // an earlier chunk of this pass gave up: the tableau is not to be touched.
  // The test is wave-uniform; waves of one workgroup may still disagree when
  // another workgroup raises the flag meanwhile, which is safe: a barrier
  // waits only for the waves that have not ended, and every later wait is
  // bounded and sees the raised flag.
  if (__builtin_amdgcn_readfirstlane(ld_relaxed(t.abort_flag))) return;
  {
    const uint32_t sk = __builtin_amdgcn_readfirstlane(chunk_skip(a.skip));
    a.qubits += sk;
    a.k -= sk;
    if (a.abort_at != kNone) a.abort_at = a.abort_at >= sk ? a.abort_at - sk : kNone;
    if (a.k == 0) return;
  }
  for (uint32_t i = tid; i < a.k; i += blockDim.x) s_q[i] = a.qubits[i];
  if (tid == 0) {
    s_abort = 0;
    s_p[0] = kNone;
    s_p[1] = kNone;
    s_par = 0;
    s_y = 0;
  }
  for (uint32_t w = tid; w < W; w += kThreads) {
    s_s0[w] = 0;
    s_s1[w] = 0;
  }
  // ---- load the owned columns: x into registers, z into LDS
  uint64_t xr[CW][L];
#pragma unroll
  for (int k = 0; k < CW; ++k) {
    const uint32_t c = wave + uint32_t(k) * kWaves;
#pragma unroll
    for (int i = 0; i < L; ++i) {
      const uint32_t w = uint32_t(i) * 64 + lane;
      const bool have = uint32_t(k) < ns && w < W;
      // every lane loads (an in-range word when it has nothing) so the loads
      // of all slots are in flight together
      const size_t at = have ? size_t(g + c * G) * t.Wp + w : 0;
      const uint64_t xv = t.X[at], zv = t.Z[at];
      xr[k][i] = have ? xv : 0ull;
      zw[(k * L + i) * 64] = have ? zv : 0ull;
    }
  }
  // Wait for these loads here: otherwise the compiler, merging them with the
  // loop's own memory operations, keeps waiting for every outstanding store
  // inside the sweep.
  __builtin_amdgcn_s_waitcnt(0);
  lds_barrier();
  // ---- the first measured column (published complete by the setup kernel)
#pragma unroll
  for (uint32_t j = 0; j < kWordsPerThread; ++j) {
    const uint32_t w = tid + j * kThreads;
    uint64_t v = 0;
    if (w < W) {
      if (!wait_published(t.pub, t.Wp, t.abort_flag, 0, w, &v)) s_abort = 1;
      s_col[0][w] = v;
    }
    wave_min_into(pivot_candidate(v, w, n, W), lane, &s_p[0]);
  }
  lds_barrier();
  if (s_abort) return;
  // this wave's share of the pivot-row support 2 s + s_x + s_z (wave-uniform)
  unsigned long long wave_sup = 0;
  uint32_t n_random = 0, n_det = 0;

#pragma unroll 1
  for (uint32_t m = 0; m < a.k; ++m) {
    // the lane index through an empty asm statement: values derived from it
    // are recomputed here each iteration instead of being hoisted out of the
    // loop and held in registers for its whole length
    uint32_t ln = lane;
    asm volatile("" : "+v"(ln));
    const uint32_t b = m & 1u;
    const uint32_t p = s_p[b];
    const uint64_t *col = s_col[b];
    const uint32_t am = s_q[m];
    const uint32_t pn = p - n, wpn = pn >> 6, wp = p >> 6;
    const uint64_t bpn = pbit(pn), bpb = pbit(p);
    const bool next = m + 1 < a.k;
    // ---- phase a: loads of slot m + 1 (this thread's word and the pivot
    // row's word, issued unconditionally so wait counts stay exact); the
    // pivot-row bits of the owned columns
    const uint64_t *nsrc = t.pub + size_t(next ? m + 1 : 0) * 2 * t.Wp;
    uint64_t f_lo[kWordsPerThread], f_hi[kWordsPerThread];
#pragma unroll
    for (uint32_t j = 0; j < kWordsPerThread; ++j) {
      const uint32_t w = tid + j * kThreads, fw = w < W ? w : 0;
      f_lo[j] = ld_relaxed64(nsrc + 2 * fw);
      f_hi[j] = ld_relaxed64(nsrc + 2 * fw + 1);
    }
    const uint32_t gw = p != kNone ? wp : 0;
    const uint64_t g_lo = ld_relaxed64(nsrc + 2 * gw), g_hi = ld_relaxed64(nsrc + 2 * gw + 1);
    // The pivot row's bits in this wave's columns (bit k = slot k): every lane
    // takes bit p of its own word (p >> 6) of every slot (no branch, so the
    // LDS reads overlap; slots past ns hold zeros), and the lane holding row
    // p hands its pair to the whole wave through a lane read.  Only this wave
    // reads them, so no barrier or LDS round trip is needed.
    uint32_t xm = 0, zm = 0;
    if (p != kNone) {
      const uint32_t ip = wp >> 6, sh = p & 63;
      uint32_t xl = 0, zl = 0;
#pragma unroll
      for (int i = 0; i < L; ++i) {
        if (uint32_t(i) != ip) continue;   // wave-uniform: one branch picks the word
#pragma unroll
        for (int k = 0; k < CW; ++k) {
          xl |= uint32_t((xr[k][i] >> sh) & 1u) << k;
          zl |= uint32_t((zw[(k * L + i) * 64] >> sh) & 1u) << k;
        }
      }
      xm = uint32_t(__builtin_amdgcn_readlane(int(xl), int(wp & 63)));
      zm = uint32_t(__builtin_amdgcn_readlane(int(zl), int(wp & 63)));
      wave_sup += uint32_t(2 * __popc(xm | zm) + __popc(xm) + __popc(zm));
    }
    // ---- phase b: sweep m, then publish a_{m+2}
    if (p != kNone) {
      uint64_t mw[L], c0[L], c1[L];
#pragma unroll
      for (int i = 0; i < L; ++i) {
        // the row mask M: rows other than p with x = 1 on the measured column
        const uint32_t w = uint32_t(i) * 64 + ln;
        mw[i] = w < W ? (w == wp ? col[w] & ~bpb : col[w]) : 0ull;
        c0[i] = c1[i] = 0;
      }
      // One wave-uniform branch per column on the pivot row's Pauli on it.
      // Rows in M that anticommute with it there contribute g = +1 or -1
      // (pivot Y: g = z - x; X: g = z(2x - 1); Z: g = x(1 - 2z)), added to
      // the mod-4 counter (c1, c0) as the two-bit value (minus, anti):
      // c1 ^= minus ^ (c0 & anti), c0 ^= anti.  Columns where the pivot row
      // is the identity are untouched.  Rows p-n and p are rewritten after.
#pragma unroll
      for (int k = 0; k < CW; ++k) {
        if (uint32_t(k) >= ns) continue;
        const uint32_t ty = ((xm >> k) & 1u) | (((zm >> k) & 1u) << 1);   // wave-uniform
        if (ty == 0) continue;
        uint64_t zz[L];
#pragma unroll
        for (int i = 0; i < L; ++i) zz[i] = zw[(k * L + i) * 64];
        if (ty == 1) {                         // pivot X: x ^= M
#pragma unroll
          for (int i = 0; i < L; ++i) {
            const uint64_t anti = zz[i] & mw[i], minus = anti & ~xr[k][i];
            c1[i] ^= minus ^ (c0[i] & anti);
            c0[i] ^= anti;
            xr[k][i] ^= mw[i];
          }
        } else if (ty == 2) {                  // pivot Z: z ^= M
#pragma unroll
          for (int i = 0; i < L; ++i) {
            const uint64_t anti = xr[k][i] & mw[i], minus = anti & zz[i];
            c1[i] ^= minus ^ (c0[i] & anti);
            c0[i] ^= anti;
            zw[(k * L + i) * 64] = zz[i] ^ mw[i];
          }
        } else {                               // pivot Y: x ^= M, z ^= M
#pragma unroll
          for (int i = 0; i < L; ++i) {
            const uint64_t anti = (xr[k][i] ^ zz[i]) & mw[i], minus = anti & xr[k][i];
            c1[i] ^= minus ^ (c0[i] & anti);
            c0[i] ^= anti;
            xr[k][i] ^= mw[i];
            zw[(k * L + i) * 64] = zz[i] ^ mw[i];
          }
        }
      }
      // the wave's counters into the workgroup sums: mod-4 addition with the
      // low plane's carry taken from the atomic XOR's old value
#pragma unroll
      for (int i = 0; i < L; ++i) {
        const uint32_t w = uint32_t(i) * 64 + ln;
        if (w < W) {
          const uint64_t old = atomicXor(&s_s0[w], (unsigned long long)c0[i]);
          atomicXor(&s_s1[w], (unsigned long long)(c1[i] ^ (old & c0[i])));
        }
      }
      // row p-n becomes the old row p; row p becomes Z on the measured
      // qubit: x in the lanes holding those words; z with lane k rewriting
      // slot k's two words
      const uint32_t ipn = wpn >> 6, ip = wp >> 6;
#pragma unroll
      for (int i = 0; i < L; ++i) {
        if (uint32_t(i) != ipn && uint32_t(i) != ip) continue;   // wave-uniform
        const uint64_t mpn = (uint32_t(i) == ipn && ln == (wpn & 63)) ? bpn : 0ull;
        const uint64_t mp = (uint32_t(i) == ip && ln == (wp & 63)) ? bpb : 0ull;
#pragma unroll
        for (int k = 0; k < CW; ++k)
          xr[k][i] = (xr[k][i] & ~(mpn | mp)) | (((xm >> k) & 1u) ? mpn : 0ull);
      }
      __builtin_amdgcn_wave_barrier();
      if (ln < ns) {
        // clear, then set, the two bits with LDS atomics that return nothing
        // (a wave's LDS operations complete in order), so no read-modify-write
        // round trip sits on the iteration's path
        unsigned long long *zk = reinterpret_cast<unsigned long long *>(
            sZ + size_t(wave) * CW * L * 64 + size_t(ln) * L * 64);   // this lane's slot
        unsigned long long *za = zk + ipn * 64 + (wpn & 63), *zb = zk + ip * 64 + (wp & 63);
        atomicAnd(za, ~bpn);
        atomicAnd(zb, ~bpb);
        atomicOr(za, ((zm >> ln) & 1u) ? bpn : 0ull);
        atomicOr(zb, g + (wave + ln * kWaves) * G == am ? bpb : 0ull);
      }
    }
    if (m + 2 < a.k) {
      // the owner publishes column a_{m+2} as it stands after measurement m
      const uint32_t a2 = s_q[m + 2];
      const uint32_t c2 = a2 / G;
      if (a2 % G == g && c2 % kWaves == wave) {
        const uint32_t k2 = c2 / kWaves;
        uint64_t *dst = t.pub + size_t(m + 2) * 2 * t.Wp;
        const uint64_t tag = uint64_t(m + 3) << 32;
        // one uniform branch per slot (a select chain over xr would make the
        // compiler index the register array dynamically)
#pragma unroll
        for (int k = 0; k < CW; ++k) {
          if (uint32_t(k) != k2) continue;
#pragma unroll
          for (int i = 0; i < L; ++i) {
            const uint32_t w = uint32_t(i) * 64 + ln;
            if (w < W) {
              st_relaxed64(dst + 2 * w, (xr[k][i] & 0xffffffffull) | tag);
              st_relaxed64(dst + 2 * w + 1, (xr[k][i] >> 32) | tag);
            }
          }
        }
      }
    }
    if (__builtin_expect(p == kNone, 0)) {
      // deterministic: per column, pairs s < t of product rows with z_s x_t
      // (prefix parity inside a word, carry across lanes and words in row
      // order) and the Y count; summed over the workgroup's columns
      uint64_t tm[L];
#pragma unroll
      for (int i = 0; i < L; ++i) tm[i] = det_word(col, n, t.NW, W, uint32_t(i) * 64 + ln);
      uint32_t ycnt = 0, par = 0;
      const uint64_t below = pbit(ln) - 1;   // lanes before this one
#pragma unroll
      for (int k = 0; k < CW; ++k) {
        if (uint32_t(k) >= ns) continue;       // wave-uniform
        uint32_t carry = 0;                    // z parity of the product rows in earlier words
#pragma unroll
        for (int i = 0; i < L; ++i) {
          const uint64_t xt = xr[k][i] & tm[i], zt = zw[(k * L + i) * 64] & tm[i];
          ycnt += uint32_t(__popcll(xt & zt));
          uint64_t pre = zt << 1;
          pre ^= pre << 1; pre ^= pre << 2; pre ^= pre << 4;
          pre ^= pre << 8; pre ^= pre << 16; pre ^= pre << 32;
          const uint64_t zb = __ballot(__popcll(zt) & 1);
          const uint32_t cin = (carry ^ uint32_t(__popcll(zb & below))) & 1u;
          par ^= (uint32_t(__popcll(xt & pre)) & 1u) ^ (cin & uint32_t(__popcll(xt)) & 1u);
          carry ^= uint32_t(__popcll(zb)) & 1u;
        }
      }
      const uint64_t pb = __ballot(par & 1u);
      for (int off = 32; off > 0; off >>= 1) ycnt += __shfl_xor(ycnt, off);
      if (ln == 0) {
        if (__popcll(pb) & 1) atomicXor(&s_par, 1u);
        if (ycnt) atomicAdd(&s_y, ycnt);
      }
    }
    lds_barrier();
    // ---- phase c: column a_{m+1} and its pivot (its words spread over the
    // threads), then
    // this workgroup's partial counters for measurement m
    if (next) {
      bool ok = true;
      uint64_t pw = 0;
      if (tid < W && p != kNone && !tagged_word(g_lo, g_hi, m + 1, &pw))
        ok = wait_published(t.pub, t.Wp, t.abort_flag, m + 1, wp, &pw);
      const uint32_t bit = uint32_t(pw >> (p & 63)) & 1u;
#pragma unroll
      for (uint32_t j = 0; j < kWordsPerThread; ++j) {
        const uint32_t w = tid + j * kThreads;
        uint64_t v = 0;
        if (w < W) {
          if (!tagged_word(f_lo[j], f_hi[j], m + 1, &v))
            ok &= wait_published(t.pub, t.Wp, t.abort_flag, m + 1, w, &v);
          if (p != kNone) {
            // measurement m's update of the column: x ^= M where the pivot
            // row has x = 1 on it; row p-n takes the pivot row's bit, row p
            // is cleared
            uint64_t mv = col[w];
            if (w == wp) mv &= ~bpb;
            if (bit) v ^= mv;
            if (w == wpn) v = bit ? (v | bpn) : (v & ~bpn);
            if (w == wp) v &= ~bpb;
          }
          s_col[b ^ 1u][w] = v;
          if (g == 0) t.SNall[size_t(m + 1) * t.Wp + w] = v;   // for the kernels after this one
        }
        wave_min_into(pivot_candidate(v, w, n, W), ln, &s_p[b ^ 1u]);
      }
      if (!ok) s_abort = 1;
    }
    if (p != kNone) {
      // read by the reduce kernel after this one: one 16-byte store per word
      uint64_t *part = t.ring + (size_t(m) * G + g) * t.Wp * 2;
      for (uint32_t w = tid; w < W; w += kThreads) {
        *reinterpret_cast<ulonglong2 *>(part + size_t(w) * 2) = make_ulonglong2(s_s0[w], s_s1[w]);
        s_s0[w] = 0;
        s_s1[w] = 0;
      }
      if (tid == 0) {
        ++n_random;
      }
    } else if (tid == 0) {
      if (s_par) atomicXor(t.detpar + m, 1u);
      if (s_y) atomicAdd(t.detY + m, s_y);
      s_par = 0;   // their last reader: cleared for the next deterministic measurement
      s_y = 0;
      ++n_det;
    }
    // every thread read s_p[b] (this measurement's pivot) before the barrier
    // that ended phase b: it becomes the target of measurement m + 2's pivot
    if (tid == 0) s_p[b] = kNone;
    if (m == a.abort_at && tid == 0) {   // injected: every workgroup stops at the same iteration
      atomicOr(t.abort_flag, 1u);
      s_abort = 1;
    }
    lds_barrier();
    if (s_abort) return;
    if (next && g == 0 && tid == 0) t.pivall[m + 1] = s_p[b ^ 1u];
  }
  // ---- write the columns back
#pragma unroll
  for (int k = 0; k < CW; ++k) {
    const uint32_t c = wave + uint32_t(k) * kWaves;
#pragma unroll
    for (int i = 0; i < L; ++i) {
      const uint32_t w = uint32_t(i) * 64 + lane;
      if (uint32_t(k) < ns && w < W) {
        t.X[size_t(g + c * G) * t.Wp + w] = xr[k][i];
        t.Z[size_t(g + c * G) * t.Wp + w] = zw[(k * L + i) * 64];
      }
    }
  }
  if (lane == 0 && wave_sup) atomicAdd(reinterpret_cast<unsigned long long *>(t.state + ST_SUPPORT), wave_sup);
  if (tid == 0) {
    if (g == 0) {
      atomicAdd(&t.state[ST_RANDOM_CNT], n_random);
      atomicAdd(&t.state[ST_DET_CNT], n_det);
    }
  }
}

// --------------------------------------------------------------- reduce ---
// c1[m][w] from the partials of all workgroups (mod-4 sum), with the check
// that the low counter plane vanishes on every updated row but p-n.
__global__ void __launch_bounds__(256) k_meas_reduce(TabDev t, uint32_t k, uint32_t G, const uint32_t *skip) {
  k -= chunk_skip(skip);
  const uint32_t m = blockIdx.x, w = blockIdx.y * blockDim.x + threadIdx.x;
  if (m >= k || w >= t.W) return;
  const uint32_t p = t.pivall[m];
  if (p == kNone) return;
  const uint64_t *part = t.ring + size_t(m) * G * t.Wp * 2 + size_t(w) * 2;
  uint64_t c0 = 0, c1 = 0;
  for (uint32_t q = 0; q < G; ++q) {
    const uint64_t b0 = part[size_t(q) * t.Wp * 2], b1 = part[size_t(q) * t.Wp * 2 + 1];
    c1 ^= b1 ^ (c0 & b0);
    c0 ^= b0;
  }
  uint64_t mw = t.SNall[size_t(m) * t.Wp + w];
  if (w == (p >> 6)) mw &= ~pbit(p);
  uint64_t bad = c0 & mw;
  const uint32_t pn = p - t.n;
  if (w == (pn >> 6)) bad &= ~pbit(pn);   // row p-n anticommutes with the pivot
  // (not counted when an x/z kernel gave up: the partials of the measurements
  // it did not reach are stale; the flag is read only here, not by every thread)
  if (bad && !ld_relaxed(t.abort_flag)) atomicAdd(&t.state[ST_ANOMALY], uint32_t(__popcll(bad)));
  t.C1all[size_t(m) * t.Wp + w] = c1;
}

// ---------------------------------------------------------------- signs ---
// One workgroup of 256 threads per shot walks the chunk in order; thread t
// holds row words t and t + 256 of the shot's sign column (W <= 512) in
// registers.  The measured column and sign-correction words of the next
// kSignAhead measurements are loaded ahead, so a step costs one LDS broadcast
// of the pivot row's sign and one barrier.  Small enough in registers and LDS
// to run beside the x/z kernel of the next chunk.  Measurement m of the
// chunk has index base + m in the call.
constexpr uint32_t kSignAhead = 4;
constexpr uint32_t kSignThreads = 256;
constexpr uint32_t kSignWords = 2;   // words per thread

__global__ void __launch_bounds__(kSignThreads) k_meas_signs(TabDev t, uint32_t k, uint32_t base, uint64_t seed,
                                                             uint64_t circuit, uint64_t shot0, uint64_t m0,
                                                             const uint32_t *skip) {
  {
    const uint32_t sk = chunk_skip(skip);
    k -= sk;
    base += sk;
  }
  // pivots, and per deterministic measurement bit 0 = the x/z parity term,
  // bits 1-2 = the Y count mod 4 (small enough to sit beside the x/z kernel)
  __shared__ uint32_t s_piv[kPersistMaxChunk];
  __shared__ uint8_t s_det[kPersistMaxChunk];
  __shared__ uint32_t s_bit[2], s_par[2], s_stop;
  const uint32_t s = blockIdx.x, tid = threadIdx.x, W = t.W, S = t.S, n = t.n;
  const uint32_t lane = tid & 63;
  // an x/z kernel gave up: nothing to finish (one read for the workgroup,
  // tested by every thread after the barrier below)
  if (tid == 0) s_stop = ld_relaxed(t.abort_flag);
  for (uint32_t i = tid; i < k; i += blockDim.x) {
    s_piv[i] = t.pivall[i];
    s_det[i] = uint8_t((t.detpar[i] & 1u) | ((t.detY[i] & 3u) << 1));
  }
  if (tid < 2) s_par[tid] = 0;
  uint64_t r[kSignWords];
#pragma unroll
  for (uint32_t j = 0; j < kSignWords; ++j) {
    const uint32_t w = tid + j * kSignThreads;
    r[j] = w < W ? t.R[size_t(w) * S + s] : 0ull;
  }
  // Loads are issued unconditionally (from word 0 of measurement 0 where
  // there is nothing to load) so every path issues the same number and the
  // compiler's wait counts stay exact.
  uint64_t am[kSignAhead][kSignWords], ac[kSignAhead][kSignWords];   // words of measurements m .. m + kSignAhead - 1
#pragma unroll
  for (uint32_t d = 0; d < kSignAhead; ++d)
#pragma unroll
    for (uint32_t j = 0; j < kSignWords; ++j) {
      const uint32_t w = tid + j * kSignThreads;
      const size_t at = (w < W && d < k) ? size_t(d) * t.Wp + w : 0;
      am[d][j] = t.SNall[at];
      ac[d][j] = t.C1all[at];
    }
  // wait for these loads here, so the loop's waits track only its own
  __builtin_amdgcn_s_waitcnt(0);
  lds_barrier();
  if (s_stop) return;
  for (uint32_t mb = 0; mb < k; mb += kSignAhead) {
#pragma unroll
    for (uint32_t d = 0; d < kSignAhead; ++d) {
      const uint32_t m = mb + d;
      const uint32_t p = m < k ? s_piv[m] : 0u;
      if (m < k) {   // uniform
        const size_t slot = size_t(base) + m;
        const uint32_t b = m & 1u;
        if (p != kNone) {
          const uint32_t wp = p >> 6, pn = p - n, wpn = pn >> 6;
          uint32_t o = 0;
          if (tid == (wp % kSignThreads)) {
            const uint64_t rw = wp / kSignThreads == 0 ? r[0] : r[1];
            s_bit[b] = uint32_t(rw >> (p & 63)) & 1u;
            o = outcome_bit(seed, circuit, shot0 + s, m0 + slot);
            t.out[slot * S + s] = uint8_t(o);
            if (s == 0) t.kind[slot] = 1;
          }
          lds_barrier();
          const uint64_t rp = s_bit[b] ? ~0ull : 0ull;
#pragma unroll
          for (uint32_t j = 0; j < kSignWords; ++j) {
            const uint32_t w = tid + j * kSignThreads;
            if (w >= W) continue;
            uint64_t mw = am[d][j];
            if (w == wp) mw &= ~pbit(p);
            uint64_t rv = r[j] ^ (mw & (ac[d][j] ^ rp));
            if (w == wpn) rv = rp ? (rv | pbit(pn)) : (rv & ~pbit(pn));
            if (w == wp) rv = o ? (rv | pbit(p)) : (rv & ~pbit(p));
            r[j] = rv;
          }
        } else {
          // deterministic: parity of the product rows' signs, then the x/z
          // terms the x/z kernel accumulated
          uint32_t par = 0;
#pragma unroll
          for (uint32_t j = 0; j < kSignWords; ++j) {
            const uint32_t w = tid + j * kSignThreads;
            if (w < W) par ^= uint32_t(__popcll(det_word(t.SNall + size_t(m) * t.Wp, n, t.NW, W, w) & r[j])) & 1u;
          }
          const uint64_t pb = __ballot(par != 0);
          if (lane == 0 && (__popcll(pb) & 1)) atomicXor(&s_par[b], 1u);
          lds_barrier();
          if (tid == 0) {
            const uint32_t dt = s_det[m];
            t.out[slot * S + s] = uint8_t(s_par[b] ^ (dt & 1u) ^ ((dt >> 2) & 1u));
            if (s == 0) {
              t.kind[slot] = 0;
              if (dt & 2u) atomicAdd(&t.state[ST_ANOMALY], 1u);   // odd Y count
            }
            s_par[b] = 0;   // next used at m + 2, after the next barrier
          }
        }
      }
      // refill this ring entry with measurement m + kSignAhead
      const uint32_t mf = m + kSignAhead;
#pragma unroll
      for (uint32_t j = 0; j < kSignWords; ++j) {
        const uint32_t w = tid + j * kSignThreads;
        const size_t at = (w < W && mf < k) ? size_t(mf) * t.Wp + w : 0;
        am[d][j] = t.SNall[at];
        ac[d][j] = t.C1all[at];
      }
    }
  }
#pragma unroll
  for (uint32_t j = 0; j < kSignWords; ++j) {
    const uint32_t w = tid + j * kSignThreads;
    if (w < W) t.R[size_t(w) * S + s] = r[j];
  }
}

// ---------------------------------------------------------------- setup ---
// Publish the first measured column (slot 0, tag 1) and the second one as it
// stands before measurement 0 (slot 1, tag 2), clear the tags of the chunk's
// other slots and the deterministic accumulators (kernel stores only, no
// memset: capture-safe).  Blocks 0 and 1 publish; every block clears a share
// of the slots.  The abort flag is left alone: it stays raised until the
// host has reported it, so later chunks of an aborted pass do nothing.
__global__ void __launch_bounds__(1024) k_meas_begin(TabDev t, const uint32_t *qubits, uint32_t k,
                                                     const uint32_t *skip) {
  __shared__ uint32_t s_p;
  {
    const uint32_t sk = chunk_skip(skip);
    qubits += sk;
    k -= sk;
    if (k == 0) return;
  }
  const uint32_t tid = threadIdx.x;
  const size_t per = 2 * size_t(t.Wp);
  for (size_t i = size_t(blockIdx.x) * blockDim.x + tid + 2 * per; i < size_t(k) * per;
       i += size_t(gridDim.x) * blockDim.x)
    t.pub[i] = 0;
  if (blockIdx.x == 1 && k > 1) {
    // slot 1: column a_1 before measurement 0 (each workgroup applies it)
    const uint64_t *c1 = t.X + size_t(qubits[1]) * t.Wp;
    for (uint32_t w = tid; w < t.Wp; w += blockDim.x) {
      const uint64_t x = w < t.W ? c1[w] : 0ull;
      t.pub[per + 2 * w] = (x & 0xffffffffull) | (2ull << 32);
      t.pub[per + 2 * w + 1] = (x >> 32) | (2ull << 32);
    }
  }
  if (blockIdx.x != 0) return;
  if (tid == 0) s_p = kNone;
  __syncthreads();
  const uint64_t *colx = t.X + size_t(qubits[0]) * t.Wp;
  for (uint32_t w = tid; w < t.Wp; w += blockDim.x) {
    uint64_t x = w < t.W ? colx[w] : 0ull;
    t.SNall[w] = x;
    t.pub[2 * w] = (x & 0xffffffffull) | (1ull << 32);
    t.pub[2 * w + 1] = (x >> 32) | (1ull << 32);
    if (w >= (t.n >> 6) && w < t.W) {
      if (w == (t.n >> 6)) x &= ~0ull << (t.n & 63);
      if (x) atomicMin(&s_p, w * 64 + uint32_t(__builtin_ctzll(x)));
    }
  }
  for (uint32_t i = tid; i < k; i += blockDim.x) {
    t.detpar[i] = 0;
    t.detY[i] = 0;
  }
  __syncthreads();
  if (tid == 0) t.pivall[0] = s_p;
}

// Launch shape of the register-resident path for n qubits (false = not
// usable): G workgroups, L row words per lane, CW = L columns per wave (8
// waves x L columns of 64 L words per workgroup: n up to 256 * 8 L >= 64 W).
bool persist_shape(uint32_t n, uint32_t num_cus, uint32_t *G, uint32_t *L, uint32_t *CW) {
  if (!persist_layout(n)) return false;
  const uint32_t W = (2 * n + 63) / 64;
  const uint32_t l = (W + 63) / 64;
  const uint32_t cw = l;
  const uint32_t gmax = num_cus < kPersistMaxGroups ? num_cus : kPersistMaxGroups;
  const uint32_t per = kWaves * cw;   // columns one workgroup holds
  const uint32_t g = (n + per - 1) / per;
  if (g > gmax) return false;
  *G = g;
  *L = l;
  *CW = cw;
  return true;
}

hipError_t launch_measure_persist(const TabDev &t, uint32_t kc, const uint32_t *dev_qubits, uint32_t k,
                                  uint64_t seed, uint64_t circuit, uint64_t shot0, uint64_t m0,
                                  int num_cus, const PersistStreams &ps, Profiler *prof, uint32_t *done,
                                  uint64_t abort_at, const BlkDev *blk, uint32_t blk_G, uint32_t blk_L) {
  *done = 0;
  uint32_t G, L, CW;
  if (!persist_shape(t.n, uint32_t(num_cus), &G, &L, &CW)) return hipErrorInvalidValue;
  if (kc == 0 || kc > kPersistMaxChunk || !t.SNall) return hipErrorInvalidValue;
  // per-chunk scratch, two sets: chunk c uses set c & 1
  TabDev tb[2] = {t, t};
  tb[1].SNall += size_t(kc) * t.Wp;
  tb[1].pivall += kc;
  tb[1].pub += size_t(kc) * 2 * t.Wp;
  tb[1].C1all += size_t(kc) * t.Wp;
  tb[1].ring += size_t(kc) * kPersistMaxGroups * t.Wp * 2;
  // a pass holds at most n measurements: set 1 serves chunks at offset kc of
  // it, so its entries end by n
  tb[1].detpar += kc;
  tb[1].detY += kc;
  const hipStream_t st = ps.main, aux = ps.aux;
  const void *fn = L == 1 ? reinterpret_cast<const void *>(k_meas_xz<1, 1>)
                 : L == 2 ? reinterpret_cast<const void *>(k_meas_xz<2, 2>)
                 : L == 3 ? reinterpret_cast<const void *>(k_meas_xz<3, 3>)
                 : L == 4 ? reinterpret_cast<const void *>(k_meas_xz<4, 4>)
                          : reinterpret_cast<const void *>(k_meas_xz<5, 5>);
  (void)CW;   // = L, fixed by the instance
  // Large chunks end the pass with a short one: the last chunk's finalize is
  // the one no later chunk hides.  (Set 1's entries at offset kc still end by
  // n: only when kc + kTail <= n.)
  constexpr uint32_t kTail = 256;
  const bool split_tail = kc >= 4 * kTail && kc + kTail <= t.n;
  uint32_t last = 0;
  for (uint32_t base = 0, c = 0, cnt = 0; base < k; base += cnt, ++c) {
    const uint32_t rem = k - base;
    cnt = rem < kc ? rem : kc;
    if (split_tail && rem > 2 * kTail && rem <= kc + kTail) cnt = rem - kTail;
    const uint32_t b = c & 1u;
    last = b;
    const TabDev &tv = tb[b];
    // set b is free once chunk c - 2's finalize is done
    hipError_t e = hipStreamWaitEvent(st, ps.ev[2 + b], 0);
    if (e != hipSuccess) return e;
    const uint32_t ab = (abort_at >= base && abort_at < uint64_t(base) + cnt) ? uint32_t(abort_at - base) : kNone;
    // the blocked pass takes the chunk's leading random measurements; the
    // kernels below do the rest (from the count it leaves in device memory)
    const uint32_t *skip = nullptr;
    if (blk) {
      if (prof) prof->begin(PK_BLOCKED, st);
      e = launch_blk_chunk(tv, blk[b], dev_qubits + base, cnt, blk_G, blk_L, ab, st);
      if (prof) prof->end(PK_BLOCKED, st);
      if (e != hipSuccess) return e;
      skip = blk[b].sync + 2;
      // its finalize needs only the blocked pass's own results: on the second
      // stream from here, during the launches below (a finalize dispatched
      // after the next chunk's blocked pass has taken the CUs waits for it)
      e = hipEventRecord(ps.ev[4 + b], st);
      if (e == hipSuccess) e = hipStreamWaitEvent(aux, ps.ev[4 + b], 0);
      if (e != hipSuccess) return e;
      if (prof) prof->begin(PK_FINAL, aux);
      e = launch_blk_finalize(tv, blk[b], cnt, base, seed, circuit, shot0, m0, blk_G, aux);
      if (prof) prof->end(PK_FINAL, aux);
      if (e != hipSuccess) return e;
    }
    // A plain launch goes to another hardware queue than the cooperative x/z
    // kernel, and each hand-off between the two is a cross-queue dependency
    // (10-20 us).  Launched cooperatively it shares the x/z kernel's queue:
    // 1.5-2.4 % faster at n = 10,000 (measured with chunks of 819), 1-5 %
    // slower from n = 256 to 8,000 (chunks of at most 341), where the
    // cooperative path's own cost per launch outweighs it; so only for the
    // large chunks of n >= 8192.
    if (prof) prof->begin(PK_SELECT, st);
    if (t.n >= 8192) {
      TabDev barg = tv;
      const uint32_t *qarg = dev_qubits + base;
      uint32_t carg = cnt;
      const uint32_t *sarg = skip;
      void *bargs[] = {&barg, &qarg, &carg, &sarg};
      e = hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k_meas_begin), dim3(64), dim3(1024), bargs, 0, st);
    } else {
      k_meas_begin<<<64, 1024, 0, st>>>(tv, dev_qubits + base, cnt, skip);
      e = hipGetLastError();
    }
    if (prof) prof->end(PK_SELECT, st);
    if (e != hipSuccess) return e;
    PersistArgs a{dev_qubits + base, cnt, G, ab, skip};
    TabDev targ = tv;
    void *args[] = {&targ, &a};
    if (prof) prof->begin(PK_SWEEP, st);
    e = hipLaunchCooperativeKernel(fn, dim3(G), dim3(kThreads), args, 0, st);
    if (prof) prof->end(PK_SWEEP, st);
    if (e != hipSuccess) return e;
    e = hipEventRecord(ps.ev[b], st);
    if (e != hipSuccess) return e;
    // finalize on the second stream, overlapping the next chunk's x/z kernel
    e = hipStreamWaitEvent(aux, ps.ev[b], 0);
    if (e != hipSuccess) return e;
    if (prof) prof->begin(PK_FINAL, aux);
    k_meas_reduce<<<dim3(cnt, (t.W + 255) / 256), 256, 0, aux>>>(tv, cnt, G, skip);
    k_meas_signs<<<t.S, kSignThreads, 0, aux>>>(tv, cnt, base, seed, circuit, shot0, m0, skip);
    if (prof) prof->end(PK_FINAL, aux);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipEventRecord(ps.ev[2 + b], aux);
    if (e != hipSuccess) return e;
    *done = base + cnt;
  }
  // the caller's stream sees the outcomes and signs only after the last finalize
  return k ? hipStreamWaitEvent(st, ps.ev[2 + last], 0) : hipSuccess;
}

}  // namespace cliff
