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
//    workgroups.  A data wave holds, for one 64-row word tile, up to CW of the
//    workgroup's columns: x bits in registers, z bits in LDS, for the whole
//    chunk, so the rowsum sweep touches no HBM.  Per measurement m the only
//    thing that travels between workgroups is the measured column a_m after
//    measurement m-1 and its pivot row p_m: the owner of a_m publishes both
//    (then a flag) as soon as it has seen measurement m-1 published, and
//    every workgroup waits for that flag only.  Each workgroup writes its
//    (c0, c1) counter pair per row word for every measurement of the chunk to
//    HBM with write-through stores.
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

constexpr uint32_t kSpinLimit = 1u << 21;   // polls before giving up (~seconds)

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
__device__ __forceinline__ void st_relaxed(uint32_t *p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed64(uint64_t *p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Destabilizer half of a published column shifted up by n rows (word w).
__device__ __forceinline__ uint64_t det_word(const uint64_t *col, uint32_t n, uint32_t NW, uint32_t W,
                                             uint32_t w) {
  if (w >= W) return 0ull;
  const uint32_t q = n >> 6, sh = n & 63;
  auto src = [&](int64_t i) -> uint64_t {
    if (i < 0 || i >= int64_t(NW)) return 0ull;
    uint64_t v = ld_relaxed64(col + i);
    if (uint32_t(i) == q && sh) v &= pbit(sh) - 1;
    return v;
  };
  const int64_t i = int64_t(w) - int64_t(q);
  uint64_t v = src(i) << sh;
  if (sh) v |= src(i - 1) >> (64 - sh);
  return v;
}

template <int CW>
__global__ void __launch_bounds__(1024) k_meas_xz(TabDev t, PersistArgs a) {
  // x bits of the owned columns live in registers, z bits in LDS
  __shared__ uint64_t sZ[16 * CW * 64];
  __shared__ uint64_t s_c0[16 * 64], s_c1[16 * 64];
  __shared__ uint32_t s_q[kPersistMaxChunk];                // this chunk's measured qubits
  __shared__ uint32_t s_xpm[16], s_zpm[16];                 // per column group: bit k = pivot-row x/z of slot k
  __shared__ uint32_t s_ztile[16 * CW], s_xtile[16 * CW];   // per column: bit = tile parity
  __shared__ uint32_t s_flag, s_pn, s_abort, s_nzw;
  __shared__ uint32_t s_par, s_y;
  const uint32_t tid = threadIdx.x, lane = tid & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const uint32_t g = blockIdx.x, G = a.G, T = a.T, NCG = a.NCG;
  const uint32_t n = t.n, W = t.W;
  const uint32_t C = g < n ? (n - g + G - 1) / G : 0;   // owned columns g, g+G, g+2G, ...
  const bool data = wave < T * NCG;
  const uint32_t tile = data ? wave % T : 0, cg = data ? wave / T : 0;
  // slots k < ns of this wave hold columns c = cg + k * NCG < C (wave-uniform)
  const uint32_t ns = data && C > cg ? (C - cg + NCG - 1) / NCG : 0;
  const uint32_t w = tile * 64 + lane;
  const bool live = data && w < W;

  for (uint32_t i = tid; i < a.k; i += blockDim.x) s_q[i] = a.qubits[i];
  // ---- load the owned columns: x into registers, z into LDS
  uint64_t xr[CW];
  uint64_t *zl = sZ + size_t(wave) * CW * 64 + lane;   // z of slot k at zl[k * 64]
#pragma unroll
  for (int k = 0; k < CW; ++k) {
    const uint32_t c = cg + uint32_t(k) * NCG;
    xr[k] = 0;
    if (data) zl[k * 64] = 0;
    if (live && uint32_t(k) < ns) {
      xr[k] = t.X[size_t(g + c * G) * t.Wp + w];
      zl[k * 64] = t.Z[size_t(g + c * G) * t.Wp + w];
    }
  }
  unsigned long long bytes_acc = 0;   // algorithmic sweep bytes of this workgroup (thread 0)
  uint32_t n_random = 0, n_det = 0;
  if (tid == 0) s_nzw = 0;

  for (uint32_t m = 0; m < a.k; ++m) {
    // ---- wait until measurement m is published; the flag word carries
    // the pivot row as p + 2 (kNone + 2 wraps to 1), so it is never zero
    uint32_t spins = 0;
    for (;;) {
      if (tid == 0) {
        s_flag = ld_relaxed(t.flags + m);
        s_abort = ld_relaxed(t.abort_flag);
        if (!s_flag && ++spins > kSpinLimit) {
          atomicOr(t.abort_flag, 1u);
          s_abort = 1;
        }
      }
      __syncthreads();
      if (s_abort) return;
      if (s_flag) break;
      __builtin_amdgcn_s_sleep(1);
      __syncthreads();
    }
    const uint32_t p = s_flag - 2u;
    const uint64_t *col = t.SNall + size_t(m) * t.Wp;
    const uint32_t am = s_q[m];
    const uint32_t a_next = m + 1 < a.k ? s_q[m + 1] : kNone;
    const bool own_next = a_next != kNone && (a_next % G) == g;
    const uint32_t cn = own_next ? a_next / G : 0;
    const uint32_t pn = p - n, wpn = pn >> 6, wp = p >> 6;
    const uint64_t bpn = pbit(pn), bpb = pbit(p);
    uint64_t mw = 0;
    if (live) {
      mw = ld_relaxed64(col + w);
      if (p != kNone && w == wp) mw &= ~bpb;
    }
    if (p != kNone && live && w == wp) {
      // the lane holding row p: pivot-row bits of this wave's slots
      uint32_t xm = 0, zm = 0;
#pragma unroll
      for (int k = 0; k < CW; ++k) {
        if (uint32_t(k) < ns) {
          xm |= uint32_t((xr[k] >> (p & 63)) & 1u) << k;
          zm |= uint32_t((zl[k * 64] >> (p & 63)) & 1u) << k;
        }
      }
      s_xpm[cg] = xm;
      s_zpm[cg] = zm;
    }
    if (tid == 0) s_pn = kNone;
    if (tid < 16 * CW) {
      s_ztile[tid] = 0;
      s_xtile[tid] = 0;
    }
    __syncthreads();
    const uint32_t xm = p != kNone ? __builtin_amdgcn_readfirstlane(s_xpm[cg]) : 0u;
    const uint32_t zm = p != kNone ? __builtin_amdgcn_readfirstlane(s_zpm[cg]) : 0u;
    // ---- publish the next measured column first (only its owner)
    const bool pub = own_next && data && (cn % NCG) == cg;
    if (pub && live) {
      const uint32_t kn = cn / NCG;
      // one uniform branch per slot (a select chain over xr would make the
      // compiler index the register array dynamically and spill it)
#pragma unroll
      for (int k = 0; k < CW; ++k) {
        if (uint32_t(k) != kn) continue;
        uint64_t x = xr[k];
        if (p != kNone) {
          const uint32_t xpj = (xm >> k) & 1u;
          uint64_t nx = xpj ? (x ^ mw) : x;
          if (w == wpn) nx = xpj ? (nx | bpn) : (nx & ~bpn);
          if (w == wp) nx &= ~bpb;
          x = nx;
        }
        st_relaxed64(t.SNall + size_t(m + 1) * t.Wp + w, x);
        uint64_t v = x;
        if (w >= (n >> 6)) {
          if (w == (n >> 6)) v &= ~0ull << (n & 63);
          if (v) atomicMin(&s_pn, w * 64 + uint32_t(__builtin_ctzll(v)));
        }
      }
    }
    if (pub) __atomic_thread_fence(__ATOMIC_RELEASE);   // each storing wave fences its own stores
    __syncthreads();
    if (own_next && tid == 0) {
      const uint32_t pnext = s_pn;
      __atomic_thread_fence(__ATOMIC_RELEASE);
      st_relaxed(t.flags + m + 1, pnext + 2u);
      t.pivall[m + 1] = pnext;   // read only by the kernels after this one
    }
    // ---- the sweep (random) or the x/z terms of the sign (deterministic)
    uint64_t c0 = 0, c1 = 0;
    if (p != kNone) {
      if (live) {
        // Branch-free per slot, with the pivot-row bits (xp, zp) of the
        // column as wave-uniform all-ones/zero masks XP, ZP.  Row i and the
        // pivot row anticommute on this column iff x zp ^ z xp; then g is +1
        // when f = x ^ (xp ? zp : z) is set and -1 otherwise (the three
        // pivot cases Y: g = z - x, X: g = z(2x - 1), Z: g = x(1 - 2z)).
#pragma unroll
        for (int k = 0; k < CW; ++k) {
          if (uint32_t(k) >= ns) continue;   // wave-uniform
          const uint32_t c = cg + uint32_t(k) * NCG;
          const uint64_t XP = 0ull - ((xm >> k) & 1u), ZP = 0ull - ((zm >> k) & 1u);
          const uint64_t x = xr[k], z = zl[k * 64];
          const uint64_t anti = ((x & ZP) ^ (z & XP)) & mw;
          const uint64_t f = x ^ ((XP & ZP) | (~XP & z));
          const uint64_t plus = anti & f, minus = anti & ~f;
          c1 ^= c0 & plus;
          c0 ^= plus;
          c1 ^= ~c0 & minus;
          c0 ^= minus;
          uint64_t nx = x ^ (XP & mw), nz = z ^ (ZP & mw);
          if (w == wpn) {
            nx = (nx & ~bpn) | (XP & bpn);
            nz = (nz & ~bpn) | (ZP & bpn);
          }
          if (w == wp) {
            nx &= ~bpb;
            nz = (g + c * G == am) ? (nz | bpb) : (nz & ~bpb);
          }
          xr[k] = nx;
          if (ZP || w == wpn || w == wp) zl[k * 64] = nz;
        }
      }
    } else {
      // deterministic: pairs s < t of product rows with z_s x_t per column
      // (prefix inside the tile, carry between tiles through LDS) and Y count
      if (tid == 0) { s_par = 0; s_y = 0; }
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
      __syncthreads();
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
      __syncthreads();
      if (tid == 0) {
        if (s_par) atomicXor(t.detpar + m, 1u);
        if (s_y) atomicAdd(t.detY + m, s_y);
      }
    }
    // ---- this workgroup's partial counters for measurement m
    if (data) {
      s_c0[wave * 64 + lane] = c0;
      s_c1[wave * 64 + lane] = c1;
      if (p != kNone && cg == 0 && live && mw) atomicAdd(&s_nzw, 1u);
    }
    __syncthreads();
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
        // algorithmic sweep bytes: per nonzero row word of the measured
        // column, x and z of every pivot-touching column read and written
        uint32_t sx = 0, sz = 0, sxz = 0;
        for (uint32_t q = 0; q < NCG; ++q) {
          const uint32_t xq = s_xpm[q], zq = s_zpm[q];
          sx += __popc(xq);
          sz += __popc(zq);
          sxz += __popc(xq | zq);
        }
        bytes_acc += 8ull * s_nzw * (2ull * sxz + sx + sz);
        ++n_random;
        s_nzw = 0;
      }
    } else if (tid == 0) {
      ++n_det;
    }
    __syncthreads();
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
    if (bytes_acc)
      atomicAdd(reinterpret_cast<unsigned long long *>(t.state + ST_SWEEP_BYTES), bytes_acc);
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
// One workgroup per shot walks the chunk in order with the shot's sign
// column in LDS.  Measurement m of the chunk has index base + m in the call.
__global__ void __launch_bounds__(256) k_meas_signs(TabDev t, uint32_t k, uint32_t base, uint64_t seed,
                                                    uint64_t circuit, uint64_t shot0, uint64_t m0) {
  __shared__ uint64_t sR[16 * 64];
  __shared__ uint32_t s_rt;
  const uint32_t s = blockIdx.x, tid = threadIdx.x, W = t.W, S = t.S, n = t.n;
  for (uint32_t w = tid; w < W; w += blockDim.x) sR[w] = t.R[size_t(w) * S + s];
  __syncthreads();
  for (uint32_t m = 0; m < k; ++m) {
    const uint32_t p = t.pivall[m];
    const uint64_t *col = t.SNall + size_t(m) * t.Wp;
    const size_t slot = size_t(base) + m;
    if (p != kNone) {
      const uint32_t rp = uint32_t(sR[p >> 6] >> (p & 63)) & 1u;
      __syncthreads();
      const uint32_t pn = p - n;
      const uint32_t o = outcome_bit(seed, circuit, shot0 + s, m0 + slot);
      for (uint32_t w = tid; w < W; w += blockDim.x) {
        uint64_t mw = col[w];
        if (w == (p >> 6)) mw &= ~pbit(p);
        const uint64_t c1 = t.C1all[size_t(m) * t.Wp + w];
        uint64_t rv = sR[w] ^ (mw & (c1 ^ (rp ? ~0ull : 0ull)));
        if (w == (pn >> 6)) rv = rp ? (rv | pbit(pn)) : (rv & ~pbit(pn));
        if (w == (p >> 6)) rv = o ? (rv | pbit(p)) : (rv & ~pbit(p));
        sR[w] = rv;
      }
      if (tid == 0) {
        t.out[slot * S + s] = uint8_t(o);
        if (s == 0) t.kind[slot] = 1;
      }
    } else {
      if (tid == 0) s_rt = 0;
      __syncthreads();
      uint32_t par = 0;
      for (uint32_t w = tid; w < W; w += blockDim.x)
        par ^= uint32_t(__popcll(det_word(col, n, t.NW, W, w) & sR[w])) & 1u;
      if (par) atomicXor(&s_rt, 1u);
      __syncthreads();
      if (tid == 0) {
        const uint32_t y = t.detY[m];
        t.out[slot * S + s] = uint8_t(s_rt ^ (t.detpar[m] & 1u) ^ ((y >> 1) & 1u));
        if (s == 0) {
          t.kind[slot] = 0;
          if (y & 1u) atomicAdd(&t.state[ST_ANOMALY], 1u);
        }
      }
    }
    __syncthreads();
  }
  for (uint32_t w = tid; w < W; w += blockDim.x) t.R[size_t(w) * S + s] = sR[w];
}

// ---------------------------------------------------------------- setup ---
// Publish the first measured column, clear flags, ring counters and
// deterministic accumulators (one kernel, no memset: capture-safe).
__global__ void __launch_bounds__(1024) k_meas_begin(TabDev t, const uint32_t *qubits, uint32_t k) {
  __shared__ uint32_t s_p;
  const uint32_t tid = threadIdx.x;
  if (tid == 0) s_p = kNone;
  __syncthreads();
  const uint64_t *colx = t.X + size_t(qubits[0]) * t.Wp;
  for (uint32_t w = tid; w < t.Wp; w += blockDim.x) {
    uint64_t x = w < t.W ? colx[w] : 0ull;
    t.SNall[w] = x;
    if (w >= (t.n >> 6) && w < t.W) {
      if (w == (t.n >> 6)) x &= ~0ull << (t.n & 63);
      if (x) atomicMin(&s_p, w * 64 + uint32_t(__builtin_ctzll(x)));
    }
  }
  for (uint32_t i = tid; i < k; i += blockDim.x) {
    t.flags[i] = 0;
    t.detpar[i] = 0;
    t.detY[i] = 0;
  }
  if (tid == 0) *t.abort_flag = 0;
  __syncthreads();
  if (tid == 0) {
    t.pivall[0] = s_p;
    t.flags[0] = s_p + 2u;   // pivot row + 2: never zero
  }
}

// Launch shape of the register-resident path for n qubits (false = not usable).
bool persist_shape(uint32_t n, uint32_t num_cus, uint32_t *G, uint32_t *T, uint32_t *NCG, uint32_t *CW) {
  if (!persist_layout(n)) return false;
  const uint32_t W = (2 * n + 63) / 64;
  const uint32_t t = (W + 63) / 64;
  const uint32_t ncg = 16 / t;
  const uint32_t gmax = num_cus < kPersistMaxGroups ? num_cus : kPersistMaxGroups;
  for (uint32_t cw : {4u, 8u, 12u, 14u}) {
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
                                  int num_cus, hipStream_t st, Profiler *prof) {
  uint32_t G, T, NCG, CW;
  if (!persist_shape(t.n, uint32_t(num_cus), &G, &T, &NCG, &CW)) return hipErrorInvalidValue;
  const uint32_t kc = persist_chunk(t.n);
  const void *fn = CW == 4 ? reinterpret_cast<const void *>(k_meas_xz<4>)
                 : CW == 8 ? reinterpret_cast<const void *>(k_meas_xz<8>)
                 : CW == 12 ? reinterpret_cast<const void *>(k_meas_xz<12>)
                            : reinterpret_cast<const void *>(k_meas_xz<14>);
  for (uint32_t base = 0; base < k; base += kc) {
    const uint32_t cnt = k - base < kc ? k - base : kc;
    if (prof) prof->begin(PK_SELECT, st);
    k_meas_begin<<<1, 1024, 0, st>>>(t, dev_qubits + base, cnt);
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
    k_meas_signs<<<t.S, 256, 0, st>>>(t, cnt, base, seed, circuit, shot0, m0);
    if (prof) prof->end(PK_FINAL, st);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace cliff
