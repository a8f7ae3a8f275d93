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
//  * x/z kernel (k_meas_xz): G workgroups of 16 waves; workgroup g owns the
//    columns j = g (mod G), so consecutive qubits belong to different
//    workgroups.  Each of the first 15 waves (data waves) holds, for one
//    64-row word tile, up to CW of the workgroup's columns: x bits in
//    registers, z bits in LDS, for the whole chunk, so the rowsum sweep
//    touches no HBM.  Between workgroups only measured columns travel: right
//    after its sweep of measurement m, the owner of a_{m+2} publishes that
//    column as it stands after measurement m, as tagged 64-bit entries (32
//    data bits and the 32-bit slot tag in one atomic store, so a reader knows
//    each entry is complete without a separate flag or fence).  One iteration
//    later every thread of every workgroup fetches one word of it into a
//    double-buffered LDS slot, and wave 15 (the loader), while the data waves
//    sweep measurement m + 1, applies measurement m + 1's update to it from
//    the measured column and pivot the workgroup already holds (x ^= M when
//    the pivot row has x = 1 there; rows p-n and p rewritten) and finds the
//    next pivot row.  Only this local step is sequential; the cross-workgroup
//    latency has a whole iteration of slack.
//    Each workgroup writes its (c0, c1) counter pair per row word for every
//    measurement of the chunk to HBM with write-through stores.
//  * reduce kernel: c1[m][w] = mod-4 sum of the partials of all workgroups.
//  * sign kernel: one workgroup per shot walks the chunk in order with that
//    shot's sign column in LDS: r ^= M & (c1 ^ r_p), rows p-n and p rewritten,
//    outcome = Philox bit; deterministic outcomes from the XOR of the product
//    rows' signs and the two x/z terms accumulated by the x/z kernel.
//
// Every wait is bounded; a timeout raises a device-wide abort flag that every
// wait checks, so all waves leave the kernel and the host reports the error.
#include "internal.h"
#include "philox.h"

namespace cliff {

constexpr uint32_t kSpinLimit = 1u << 20;   // polling rounds before giving up (~seconds)
constexpr uint32_t kDataWaves = 15;         // wave 15 is the loader

struct PersistArgs {
  const uint32_t *qubits;   // device, this chunk's k entries
  uint32_t k, G, T, NCG;
};

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

// Workgroup barrier ordering LDS only.  In the x/z and sign kernels the
// waves of a workgroup share data through LDS alone (global memory is read
// or written per thread, or exchanged between workgroups with atomics), so
// global loads and stores may stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
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

// One thread per row word: wait for the tagged entries of word w of
// published slot j and return the word; false when the wait gave up or
// another workgroup raised the abort flag.
__device__ __forceinline__ bool fetch_published(const TabDev &t, uint32_t j, uint32_t w, uint64_t *out) {
  const uint64_t *src = t.pub + size_t(j) * 2 * t.Wp + 2 * w;
  const uint64_t tag = uint64_t(j + 1) << 32, hi_mask = ~0xffffffffull;
  uint64_t lo = ld_relaxed64(src), hi = ld_relaxed64(src + 1);
  uint32_t spins = 0;
  while ((lo & hi_mask) != tag || (hi & hi_mask) != tag) {
    if (__hip_atomic_load(t.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
    if (++spins > kSpinLimit) {
      atomicOr(t.abort_flag, 1u);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
    lo = ld_relaxed64(src);
    hi = ld_relaxed64(src + 1);
  }
  *out = (lo & 0xffffffffull) | (hi << 32);
  return true;
}

// Loader wave: col holds a fetched slot.  When pm != kNone the slot is the
// column as it stood before the measurement whose measured column is colm
// and pivot row pm: its update is applied in place (x ^= M if the pivot row
// has x = 1 on this column, M = colm without row pm; row pm - n takes the
// pivot row's bit, row pm is cleared).  Returns the pivot row of the result:
// the smallest stabilizer row with x = 1, or kNone.
__device__ uint32_t apply_published(uint64_t *col, const uint64_t *colm, uint32_t pm, uint32_t W,
                                    uint32_t n, uint32_t lane) {
  constexpr uint32_t kU = 2;   // words per lane in flight
  uint32_t bit = 0;
  if (pm != kNone) bit = uint32_t(col[pm >> 6] >> (pm & 63)) & 1u;   // read before any lane writes
  __builtin_amdgcn_wave_barrier();
  const uint32_t pn = pm - n;
  uint32_t best = kNone;   // wave-uniform: words are visited in increasing order
  for (uint32_t w0 = 0; w0 < W; w0 += 64 * kU) {
    uint64_t v[kU], mw[kU];
#pragma unroll
    for (uint32_t u = 0; u < kU; ++u) {
      const uint32_t w = w0 + u * 64 + lane;
      v[u] = w < W ? col[w] : 0ull;
      mw[u] = (w < W && pm != kNone && bit) ? colm[w] : 0ull;
    }
#pragma unroll
    for (uint32_t u = 0; u < kU; ++u) {
      const uint32_t w = w0 + u * 64 + lane;
      uint64_t x = v[u];
      if (w < W && pm != kNone) {
        uint64_t m = mw[u];
        if (w == (pm >> 6)) m &= ~pbit(pm);
        x ^= m;
        if (w == (pn >> 6)) x = bit ? (x | pbit(pn)) : (x & ~pbit(pn));
        if (w == (pm >> 6)) x &= ~pbit(pm);
        col[w] = x;
      }
      uint64_t sv = (w < W && w >= (n >> 6)) ? x : 0ull;
      if (w == (n >> 6)) sv &= ~0ull << (n & 63);
      const uint64_t bal = __ballot(sv != 0ull);
      if (best == kNone && bal) {
        const uint32_t l = uint32_t(__builtin_ctzll(bal));
        const uint64_t hv = __shfl(sv, int(l));
        best = (w0 + u * 64 + l) * 64 + uint32_t(__builtin_ctzll(hv));
      }
    }
  }
  return best;
}

template <int CW>
__global__ void __launch_bounds__(1024) k_meas_xz(TabDev t, PersistArgs a) {
  // x bits of the owned columns live in registers, z bits in LDS
  __shared__ uint64_t sZ[kDataWaves * CW * 64];
  __shared__ uint64_t s_c0[kDataWaves * 64], s_c1[kDataWaves * 64];
  __shared__ uint64_t s_col[2][kPersistMaxWp];          // column of measurement m in s_col[m & 1]
  __shared__ uint32_t s_q[kPersistMaxChunk];            // this chunk's measured qubits
  __shared__ uint32_t s_p[2];                           // pivot row of measurement m in s_p[m & 1]
  __shared__ uint32_t s_xpm[2][kDataWaves], s_zpm[2][kDataWaves];   // per column group: bit k = slot k
  __shared__ uint32_t s_ztile[kDataWaves * CW], s_xtile[kDataWaves * CW];   // per column: bit = tile parity
  __shared__ uint32_t s_abort, s_par, s_y, s_acc[2];
  const uint32_t tid = threadIdx.x, lane = tid & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const uint32_t g = blockIdx.x, G = a.G, T = a.T, NCG = a.NCG;
  const uint32_t n = t.n, W = t.W;
  const uint32_t C = g < n ? (n - g + G - 1) / G : 0;   // owned columns g, g+G, g+2G, ...
  const bool data = wave < T * NCG;
  const bool loader = wave == kDataWaves;
  const uint32_t tile = data ? wave % T : 0, cg = data ? wave / T : 0;
  // slots k < ns of this wave hold columns c = cg + k * NCG < C (wave-uniform)
  const uint32_t ns = data && C > cg ? (C - cg + NCG - 1) / NCG : 0;
  const uint32_t w = tile * 64 + lane;
  const bool live = data && w < W;

  for (uint32_t i = tid; i < a.k; i += blockDim.x) s_q[i] = a.qubits[i];
  if (tid == 0) {
    s_abort = 0;
    s_acc[0] = 0;
    s_acc[1] = 0;
  }
  // ---- load the owned columns: x into registers, z into LDS
  uint64_t xr[CW];
  uint64_t *zl = sZ + size_t(data ? wave : 0) * CW * 64 + lane;   // z of slot k at zl[k * 64]
#pragma unroll
  for (int k = 0; k < CW; ++k) {
    const uint32_t c = cg + uint32_t(k) * NCG;
    const bool have = live && uint32_t(k) < ns;
    // every lane loads (an in-range word when it has no column) so the loads
    // of all slots are in flight together
    const size_t at = have ? size_t(g + c * G) * t.Wp + w : 0;
    const uint64_t xv = t.X[at], zv = t.Z[at];
    xr[k] = have ? xv : 0ull;
    if (data) zl[k * 64] = have ? zv : 0ull;
  }
  // Wait for these loads here: otherwise the compiler, merging them with the
  // loop's own memory operations, keeps waiting for every outstanding store
  // inside the sweep.
  __builtin_amdgcn_s_waitcnt(0);
  lds_barrier();
  if (tid < W) {
    uint64_t v;
    if (fetch_published(t, 0, tid, &v)) s_col[0][tid] = v;
    else s_abort = 1;
  }
  lds_barrier();
  if (loader) {
    const uint32_t p0 = apply_published(s_col[0], nullptr, kNone, W, n, lane);
    if (lane == 0) s_p[0] = p0;
  }
  lds_barrier();
  if (s_abort) return;
  unsigned long long sup_acc = 0;     // this workgroup's share of 2 s + s_x + s_z (thread 0)
  uint32_t n_random = 0, n_det = 0;
  uint64_t pf_lo = 0, pf_hi = 0;      // this thread's entries of slot m + 1, loaded early

  for (uint32_t m = 0; m < a.k; ++m) {
    const uint32_t b = m & 1u;
    const uint32_t p = s_p[b];
    const uint64_t *col = s_col[b];
    const uint32_t am = s_q[m];
    const uint32_t pn = p - n, wpn = pn >> 6, wp = p >> 6;
    const uint64_t bpn = pbit(pn), bpb = pbit(p);
    // ---- phase 1: fetch slot m + 1 (one word per thread); the row mask M and
    // the pivot-row bits of the owned columns
    if (m + 1 < a.k && tid < W) {
      const uint64_t tag = uint64_t(m + 2) << 32, hi_mask = ~0xffffffffull;
      uint64_t v;
      if ((pf_lo & hi_mask) == tag && (pf_hi & hi_mask) == tag)
        s_col[b ^ 1u][tid] = (pf_lo & 0xffffffffull) | (pf_hi << 32);
      else if (fetch_published(t, m + 1, tid, &v))
        s_col[b ^ 1u][tid] = v;
      else
        s_abort = 1;
    }
    uint64_t mw = 0;
    if (live) {
      mw = col[w];
      if (p != kNone && w == wp) mw &= ~bpb;
    }
    if (p != kNone && live && w == wp) {
      uint32_t xm = 0, zm = 0;
#pragma unroll
      for (int k = 0; k < CW; ++k) {
        if (uint32_t(k) < ns) {
          xm |= uint32_t((xr[k] >> (p & 63)) & 1u) << k;
          zm |= uint32_t((zl[k * 64] >> (p & 63)) & 1u) << k;
        }
      }
      s_xpm[b][cg] = xm;
      s_zpm[b][cg] = zm;
      atomicAdd(&s_acc[b], uint32_t(2 * __popc(xm | zm) + __popc(xm) + __popc(zm)));
    }
    if (p == kNone) {
      if (tid < kDataWaves * CW) {
        s_ztile[tid] = 0;
        s_xtile[tid] = 0;
      }
      if (tid == 0) {
        s_par = 0;
        s_y = 0;
      }
    }
    lds_barrier();
    if (s_abort) return;
    // ---- phase 2: sweep m, then publish a_{m+2}; the loader applies
    // measurement m to the fetched column a_{m+1}
    const uint32_t xm = p != kNone && data ? __builtin_amdgcn_readfirstlane(s_xpm[b][cg]) : 0u;
    const uint32_t zm = p != kNone && data ? __builtin_amdgcn_readfirstlane(s_zpm[b][cg]) : 0u;
    uint64_t c0 = 0, c1 = 0;
    if (p != kNone) {
      if (live) {
        // One wave-uniform branch per slot on the pivot row's Pauli on that
        // column.  Rows in M that anticommute with it there contribute
        // g = +1 or -1 (pivot Y: g = z - x; X: g = z(2x - 1); Z: g = x(1 - 2z)),
        // added to the mod-4 counter (c1, c0) as the two-bit value
        // (minus, anti): c1 ^= minus ^ (c0 & anti), c0 ^= anti.  Columns where
        // the pivot row is the identity are untouched.  Rows p-n and p are
        // rewritten afterwards.
#pragma unroll
        for (int k = 0; k < CW; ++k) {
          if (uint32_t(k) >= ns) continue;
          const uint32_t ty = ((xm >> k) & 1u) | (((zm >> k) & 1u) << 1);   // wave-uniform
          if (ty == 0) continue;
          const uint64_t x = xr[k], z = zl[k * 64];
          if (ty == 1) {                       // pivot X: x ^= M
            const uint64_t anti = z & mw, minus = anti & ~x;
            c1 ^= minus ^ (c0 & anti);
            c0 ^= anti;
            xr[k] = x ^ mw;
          } else if (ty == 2) {                // pivot Z: z ^= M
            const uint64_t anti = x & mw, minus = anti & z;
            c1 ^= minus ^ (c0 & anti);
            c0 ^= anti;
            zl[k * 64] = z ^ mw;
          } else {                             // pivot Y: x ^= M, z ^= M
            const uint64_t anti = (x ^ z) & mw, minus = anti & x;
            c1 ^= minus ^ (c0 & anti);
            c0 ^= anti;
            xr[k] = x ^ mw;
            zl[k * 64] = z ^ mw;
          }
        }
        // row p-n becomes the old row p; row p becomes Z on the measured
        // qubit (only the waves holding those two words): x in the lane
        // holding the word, branch-free over the slots; z with lane k
        // rewriting slot k's word of that lane
        if (tile == (wpn >> 6) || tile == (wp >> 6)) {
          const uint64_t mpn = w == wpn ? bpn : 0ull, mp = w == wp ? bpb : 0ull;
#pragma unroll
          for (int k = 0; k < CW; ++k)
            if (uint32_t(k) < ns) xr[k] = (xr[k] & ~(mpn | mp)) | (((xm >> k) & 1u) ? mpn : 0ull);
          __builtin_amdgcn_wave_barrier();
          if (lane < ns) {
            uint64_t *zk = sZ + size_t(wave) * CW * 64 + lane * 64;
            if (tile == (wpn >> 6)) {
              uint64_t &zw = zk[wpn & 63];
              zw = ((zm >> lane) & 1u) ? (zw | bpn) : (zw & ~bpn);
            }
            if (tile == (wp >> 6)) {
              uint64_t &zw = zk[wp & 63];
              zw = (g + (cg + lane * NCG) * G == am) ? (zw | bpb) : (zw & ~bpb);
            }
          }
        }
      }
    }
    if (m + 2 < a.k && live) {
      // the owner publishes column a_{m+2} as it stands after measurement m
      const uint32_t a2 = s_q[m + 2];
      const uint32_t c2 = a2 / G;
      if (a2 % G == g && c2 % NCG == cg) {
        const uint32_t k2 = c2 / NCG;
        uint64_t *dst = t.pub + size_t(m + 2) * 2 * t.Wp + 2 * w;
        const uint64_t tag = uint64_t(m + 3) << 32;
        // one uniform branch per slot (a select chain over xr would make the
        // compiler index the register array dynamically)
#pragma unroll
        for (int k = 0; k < CW; ++k) {
          if (uint32_t(k) != k2) continue;
          st_relaxed64(dst, (xr[k] & 0xffffffffull) | tag);
          st_relaxed64(dst + 1, (xr[k] >> 32) | tag);
        }
      }
    }
    if (loader && m + 1 < a.k) {
      const uint32_t pnext = apply_published(s_col[b ^ 1u], col, p, W, n, lane);
      if (lane == 0) s_p[b ^ 1u] = pnext;
      if (g == 0) {
        // for the reduce and sign kernels after this one
        for (uint32_t ww = lane; ww < W; ww += 64) t.SNall[size_t(m + 1) * t.Wp + ww] = s_col[b ^ 1u][ww];
        if (lane == 0) t.pivall[m + 1] = pnext;
      }
    }
    if (p == kNone) {
      // deterministic: pairs s < t of product rows with z_s x_t per column
      // (prefix inside the tile, carry between tiles through LDS) and Y count
      const uint64_t Tm = live ? det_word(col, n, t.NW, W, w) : 0ull;
      uint32_t ycnt = 0, par = 0;
      if (data) {
#pragma unroll
        for (int k = 0; k < CW; ++k) {
          if (uint32_t(k) >= ns) continue;   // uniform across the wave
          const uint32_t c = cg + uint32_t(k) * NCG;
          const uint64_t xt = xr[k] & Tm, zt = zl[k * 64] & Tm;
          ycnt += uint32_t(__popcll(xt & zt));
          uint64_t pre = zt << 1;
          pre ^= pre << 1; pre ^= pre << 2; pre ^= pre << 4;
          pre ^= pre << 8; pre ^= pre << 16; pre ^= pre << 32;
          const uint64_t zb = __ballot(__popcll(zt) & 1);
          const uint64_t xb = __ballot(__popcll(xt) & 1);
          const uint32_t cin = uint32_t(__popcll(zb & (pbit(lane) - 1))) & 1u;
          par ^= (uint32_t(__popcll(xt & pre)) & 1u) ^ (cin & uint32_t(__popcll(xt)) & 1u);
          if (lane == 0) {
            if (__popcll(zb) & 1) atomicOr(&s_ztile[c], 1u << tile);
            if (__popcll(xb) & 1) atomicOr(&s_xtile[c], 1u << tile);
          }
        }
      }
      const uint64_t pb = __ballot(par & 1u);
      for (int off = 32; off > 0; off >>= 1) ycnt += __shfl_xor(ycnt, off);
      lds_barrier();
      if (lane == 0 && data) {
        uint32_t extra = __popcll(pb) & 1u;
        // carry into this tile from the z parities of the tiles before it
        for (uint32_t k = 0; k < ns; ++k) {
          const uint32_t c = cg + k * NCG;
          const uint32_t carry = uint32_t(__popc(s_ztile[c] & ((1u << tile) - 1u))) & 1u;
          extra ^= carry & (s_xtile[c] >> tile) & 1u;
        }
        if (extra) atomicXor(&s_par, 1u);
        if (ycnt) atomicAdd(&s_y, ycnt);
      }
      lds_barrier();
      if (tid == 0) {
        if (s_par) atomicXor(t.detpar + m, 1u);
        if (s_y) atomicAdd(t.detY + m, s_y);
      }
    }
    // ---- this workgroup's partial counters for measurement m
    if (p != kNone && data) {
      s_c0[wave * 64 + lane] = c0;
      s_c1[wave * 64 + lane] = c1;
    }
    lds_barrier();
    // ---- phase 3: load this thread's entries of slot m + 2 early (its owner
    // publishes it during iteration m; checked at the next iteration's top),
    // combine the column groups and write the partials
    if (m + 2 < a.k && tid < W) {
      const uint64_t *src = t.pub + size_t(m + 2) * 2 * t.Wp + 2 * tid;
      pf_lo = ld_relaxed64(src);
      pf_hi = ld_relaxed64(src + 1);
    }
    if (p != kNone) {
      uint64_t *part = t.ring + (size_t(m) * G + g) * t.Wp * 2;
      for (uint32_t ww = tid; ww < W; ww += blockDim.x) {
        const uint32_t tl = ww / 64, ln = ww % 64;
        uint64_t a0 = 0, a1 = 0;
        for (uint32_t gg = 0; gg < NCG; ++gg) {
          const uint32_t wv = gg * T + tl;
          const uint64_t b0 = s_c0[wv * 64 + ln], b1 = s_c1[wv * 64 + ln];
          a1 ^= b1 ^ (a0 & b0);
          a0 ^= b0;
        }
        // read by the reduce kernel after this one: write-through, no fence
        st_relaxed64(part + size_t(ww) * 2, a0);
        st_relaxed64(part + size_t(ww) * 2 + 1, a1);
      }
      if (tid == 0) {
        // pivot-row support over this workgroup's columns: 2 s + s_x + s_z
        sup_acc += s_acc[b];
        ++n_random;
        s_acc[b] = 0;
      }
    } else if (tid == 0) {
      ++n_det;
    }
  }
  // ---- write the columns back
#pragma unroll
  for (int k = 0; k < CW; ++k) {
    const uint32_t c = cg + uint32_t(k) * NCG;
    if (live && uint32_t(k) < ns) {
      t.X[size_t(g + c * G) * t.Wp + w] = xr[k];
      t.Z[size_t(g + c * G) * t.Wp + w] = zl[k * 64];
    }
  }
  if (tid == 0) {
    if (sup_acc) atomicAdd(reinterpret_cast<unsigned long long *>(t.state + ST_SUPPORT), sup_acc);
    if (g == 0) {
      atomicAdd(&t.state[ST_RANDOM_CNT], n_random);
      atomicAdd(&t.state[ST_DET_CNT], n_det);
    }
  }
}

// --------------------------------------------------------------- reduce ---
// c1[m][w] from the partials of all workgroups (mod-4 sum), with the check
// that the low counter plane vanishes on every updated row but p-n.
__global__ void __launch_bounds__(256) k_meas_reduce(TabDev t, uint32_t k, uint32_t G) {
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
  if (bad) atomicAdd(&t.state[ST_ANOMALY], uint32_t(__popcll(bad)));
  t.C1all[size_t(m) * t.Wp + w] = c1;
}

// ---------------------------------------------------------------- signs ---
// One workgroup per shot walks the chunk in order; thread w holds row word w
// of the shot's sign column (W <= 960) in a register.  The measured column
// and sign-correction words of the next kSignAhead measurements are loaded
// ahead, so a step costs one LDS broadcast of the pivot row's sign and one
// barrier.  Measurement m of the chunk has index base + m in the call.
constexpr uint32_t kSignAhead = 8;

__global__ void __launch_bounds__(1024) k_meas_signs(TabDev t, uint32_t k, uint32_t base, uint64_t seed,
                                                     uint64_t circuit, uint64_t shot0, uint64_t m0) {
  __shared__ uint32_t s_piv[kPersistMaxChunk], s_dp[kPersistMaxChunk], s_dy[kPersistMaxChunk];
  __shared__ uint32_t s_bit[2], s_par[2];
  const uint32_t s = blockIdx.x, tid = threadIdx.x, W = t.W, S = t.S, n = t.n;
  const uint32_t lane = tid & 63;
  const bool own = tid < W;
  for (uint32_t i = tid; i < k; i += blockDim.x) {
    s_piv[i] = t.pivall[i];
    s_dp[i] = t.detpar[i];
    s_dy[i] = t.detY[i];
  }
  if (tid < 2) s_par[tid] = 0;
  uint64_t r = own ? t.R[size_t(tid) * S + s] : 0ull;
  uint64_t am[kSignAhead], ac[kSignAhead];   // words of measurements m .. m + kSignAhead - 1
  // Loads are issued unconditionally (from word 0 of measurement 0 where
  // there is nothing to load) so every path issues the same number and the
  // compiler's wait counts stay exact.
#pragma unroll
  for (uint32_t d = 0; d < kSignAhead; ++d) {
    const size_t at = (own && d < k) ? size_t(d) * t.Wp + tid : 0;
    am[d] = t.SNall[at];
    ac[d] = t.C1all[at];
  }
  // wait for these loads here, so the loop's waits track only its own
  __builtin_amdgcn_s_waitcnt(0);
  lds_barrier();
  for (uint32_t mb = 0; mb < k; mb += kSignAhead) {
#pragma unroll
    for (uint32_t d = 0; d < kSignAhead; ++d) {
      const uint32_t m = mb + d;
      const uint32_t p = m < k ? s_piv[m] : 0u;
      if (m < k) {   // uniform
        const size_t slot = size_t(base) + m;
        const uint32_t b = m & 1u;
        if (p != kNone) {
          const uint32_t wp = p >> 6, pn = p - n;
          uint32_t o = 0;
          if (tid == wp) {
            s_bit[b] = uint32_t(r >> (p & 63)) & 1u;
            o = outcome_bit(seed, circuit, shot0 + s, m0 + slot);
            t.out[slot * S + s] = uint8_t(o);
            if (s == 0) t.kind[slot] = 1;
          }
          lds_barrier();
          const uint64_t rp = s_bit[b] ? ~0ull : 0ull;
          if (own) {
            uint64_t mw = am[d];
            if (tid == wp) mw &= ~pbit(p);
            r ^= mw & (ac[d] ^ rp);
            if (tid == (pn >> 6)) r = rp ? (r | pbit(pn)) : (r & ~pbit(pn));
            if (tid == wp) r = o ? (r | pbit(p)) : (r & ~pbit(p));
          }
        } else {
          // deterministic: parity of the product rows' signs, then the x/z
          // terms the x/z kernel accumulated
          uint32_t par = 0;
          if (own) par = uint32_t(__popcll(det_word(t.SNall + size_t(m) * t.Wp, n, t.NW, W, tid) & r)) & 1u;
          const uint64_t pb = __ballot(par != 0);
          if (lane == 0 && (__popcll(pb) & 1)) atomicXor(&s_par[b], 1u);
          lds_barrier();
          if (tid == 0) {
            const uint32_t y = s_dy[m];
            t.out[slot * S + s] = uint8_t(s_par[b] ^ (s_dp[m] & 1u) ^ ((y >> 1) & 1u));
            if (s == 0) {
              t.kind[slot] = 0;
              if (y & 1u) atomicAdd(&t.state[ST_ANOMALY], 1u);
            }
            s_par[b] = 0;   // next used at m + 2, after the next barrier
          }
        }
      }
      // refill this ring entry with measurement m + kSignAhead
      const uint32_t mf = m + kSignAhead;
      const size_t at = (own && mf < k) ? size_t(mf) * t.Wp + tid : 0;
      am[d] = t.SNall[at];
      ac[d] = t.C1all[at];
    }
  }
  if (own) t.R[size_t(tid) * S + s] = r;
}

// ---------------------------------------------------------------- setup ---
// Publish the first measured column (slot 0, tag 1) and the second one as it
// stands before measurement 0 (slot 1, tag 2), clear the tags of the chunk's
// other slots, the deterministic accumulators and the abort flag (kernel
// stores only, no memset: capture-safe).  Blocks 0 and 1 publish; every
// block clears a share of the slots.
__global__ void __launch_bounds__(1024) k_meas_begin(TabDev t, const uint32_t *qubits, uint32_t k) {
  __shared__ uint32_t s_p;
  const uint32_t tid = threadIdx.x;
  const size_t per = 2 * size_t(t.Wp);
  for (size_t i = size_t(blockIdx.x) * blockDim.x + tid + 2 * per; i < size_t(k) * per;
       i += size_t(gridDim.x) * blockDim.x)
    t.pub[i] = 0;
  if (blockIdx.x == 1 && k > 1) {
    // slot 1: column a_1 before measurement 0 (the loader applies it)
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
  if (tid == 0) *t.abort_flag = 0;
  __syncthreads();
  if (tid == 0) t.pivall[0] = s_p;
}

// Launch shape of the register-resident path for n qubits (false = not usable).
bool persist_shape(uint32_t n, uint32_t num_cus, uint32_t *G, uint32_t *T, uint32_t *NCG, uint32_t *CW) {
  if (!persist_layout(n)) return false;
  const uint32_t W = (2 * n + 63) / 64;
  const uint32_t t = (W + 63) / 64;
  const uint32_t ncg = kDataWaves / t;          // column groups of t data waves
  const uint32_t gmax = num_cus < kPersistMaxGroups ? num_cus : kPersistMaxGroups;
  for (uint32_t cw : {4u, 8u, 12u, 14u, 16u}) {
    const uint32_t per = ncg * cw;              // columns one workgroup can hold
    uint32_t g = (n + per - 1) / per;
    if (g > gmax) continue;
    if (g < gmax / 4) g = gmax / 4;             // enough waves for the sweep
    if (g < 1) g = 1;
    *G = g;
    *T = t;
    *NCG = ncg;
    *CW = cw;
    return true;
  }
  return false;
}

hipError_t launch_measure_persist(const TabDev &t, const uint32_t *dev_qubits, uint32_t k,
                                  uint64_t seed, uint64_t circuit, uint64_t shot0, uint64_t m0,
                                  int num_cus, hipStream_t st, Profiler *prof, uint32_t *done) {
  *done = 0;
  uint32_t G, T, NCG, CW;
  if (!persist_shape(t.n, uint32_t(num_cus), &G, &T, &NCG, &CW)) return hipErrorInvalidValue;
  const uint32_t kc = persist_chunk(t.n);
  const void *fn = CW == 4 ? reinterpret_cast<const void *>(k_meas_xz<4>)
                 : CW == 8 ? reinterpret_cast<const void *>(k_meas_xz<8>)
                 : CW == 12 ? reinterpret_cast<const void *>(k_meas_xz<12>)
                 : CW == 14 ? reinterpret_cast<const void *>(k_meas_xz<14>)
                            : reinterpret_cast<const void *>(k_meas_xz<16>);
  for (uint32_t base = 0; base < k; base += kc) {
    const uint32_t cnt = k - base < kc ? k - base : kc;
    if (prof) prof->begin(PK_SELECT, st);
    k_meas_begin<<<64, 1024, 0, st>>>(t, dev_qubits + base, cnt);
    if (prof) prof->end(PK_SELECT, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    PersistArgs a{dev_qubits + base, cnt, G, T, NCG};
    TabDev tv = t;
    void *args[] = {&tv, &a};
    if (prof) prof->begin(PK_SWEEP, st);
    e = hipLaunchCooperativeKernel(fn, dim3(G), dim3(1024), args, 0, st);
    if (prof) prof->end(PK_SWEEP, st);
    if (e != hipSuccess) return e;
    if (prof) prof->begin(PK_FINAL, st);
    k_meas_reduce<<<dim3(cnt, (t.W + 255) / 256), 256, 0, st>>>(t, cnt, G);
    k_meas_signs<<<t.S, 1024, 0, st>>>(t, cnt, base, seed, circuit, shot0, m0);
    if (prof) prof->end(PK_FINAL, st);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    *done = base + cnt;
  }
  return hipSuccess;
}

}  // namespace cliff
