// Z-measurement of one qubit on an HBM-resident tableau (multi-kernel path).
//
// Method (paper Sec. 2, after Aaronson & Gottesman 2004):
//   random branch  -- some stabilizer row p has x_pa = 1 (take the smallest):
//     every other row i with x_ia = 1 becomes row_p * row_i ("rowsum"), whose
//     sign is r_i ^ r_p ^ (sum_j g(p_j, i_j) / 2 mod 2); row p-n takes old row
//     p; row p becomes +-Z_a with a fresh random sign, which is the outcome.
//   deterministic branch -- no such row: the outcome is the sign of the
//     product of the stabilizers n+i with x_ia = 1; the tableau is unchanged.
//
// Bit-level form used here: M = column x_a without bit p is the set of rows to
// update.  For each column j where the pivot is not I, the 64 rows of a word
// get g in {+1, -1, 0} from (x_pj, z_pj) and the row bits, accumulated in a
// bit-sliced 2-bit counter (c0, c1) per row; x_j ^= M if x_pj, z_j ^= M if
// z_pj.  With every updated row commuting with the pivot the counter ends even
// and its high plane c1 is the sign correction.  Row rewrites of p-n and p are
// folded into the same sweep, so each column word is read and written once.
//
// Deterministic sign in closed form: with T the product rows, each row written
// (-1)^r i^(x.z) X^x Z^z, the ordered product is
//   (-1)^(sum_T r + sum_j sum_{s<t in T} z_sj x_tj) * i^(sum_T x.z) * (+-Z_a),
// so outcome = XOR_T r  ^  XOR_j parity(pairs s<t with z_sj x_tj)  ^  (Y/2 mod 2)
// where Y = number of (row, column) entries with x = z = 1 (always even).
#include "internal.h"
#include "philox.h"

namespace cliff {

// ---------------------------------------------------------------- select ---
// One block: pivot search (smallest stabilizer row with x_a = 1), snapshot of
// the update mask M, packed pivot row and packed pivot signs; or, when
// deterministic, the product-row mask T (stabilizer rows n+i with x_ia = 1).
__global__ void __launch_bounds__(1024) k_select(TabDev t, uint32_t a, uint32_t slot) {
  __shared__ uint32_t s_p, s_nzw, s_sx, s_sz, s_s;
  const uint32_t tid = threadIdx.x, bd = blockDim.x;
  if (tid == 0) {
    s_p = kNone;
    s_nzw = s_sx = s_sz = s_s = 0;
  }
  __syncthreads();
  const uint64_t *colX = t.X + size_t(a) * t.Wp;
  const uint32_t n = t.n;
  const uint32_t w0 = n >> 6;
  for (uint32_t w = w0 + tid; w < t.W; w += bd) {
    uint64_t v = colX[w];
    if (w == w0) v &= ~0ull << (n & 63);
    if (v) atomicMin(&s_p, w * 64 + uint32_t(__builtin_ctzll(v)));
  }
  __syncthreads();
  const uint32_t p = s_p;
  if (p != kNone) {
    const uint32_t wp = p >> 6, bp = p & 63;
    for (uint32_t w = tid; w < t.Wp; w += bd) {
      uint64_t v = w < t.W ? colX[w] : 0ull;
      if (w == wp) v &= ~(1ull << bp);
      t.M[w] = v;
      if (v) atomicAdd(&s_nzw, 1u);
    }
    for (uint32_t j = tid; j < t.NW * 64; j += bd) {   // 64 consecutive columns per wave
      uint32_t xb = 0, zb = 0;
      if (j < n) {
        xb = uint32_t(t.X[size_t(j) * t.Wp + wp] >> bp) & 1u;
        zb = uint32_t(t.Z[size_t(j) * t.Wp + wp] >> bp) & 1u;
      }
      const uint64_t bx = __ballot(xb), bz = __ballot(zb);
      if ((tid & 63) == 0) {
        t.xp[j >> 6] = bx;
        t.zp[j >> 6] = bz;
        atomicAdd(&s_sx, uint32_t(__popcll(bx)));
        atomicAdd(&s_sz, uint32_t(__popcll(bz)));
        atomicAdd(&s_s, uint32_t(__popcll(bx | bz)));
      }
    }
    for (uint32_t s = tid; s < t.SW * 64; s += bd) {
      const uint32_t rb = s < t.S ? uint32_t(t.R[size_t(wp) * t.S + s] >> bp) & 1u : 0u;
      const uint64_t b = __ballot(rb);
      if ((tid & 63) == 0) t.rp[s >> 6] = b;
    }
  } else {
    // T = (destabilizer half of column a) shifted up by n rows
    const uint32_t q = n >> 6, sh = n & 63;
    auto src = [&](int64_t i) -> uint64_t {
      if (i < 0 || i >= int64_t(t.NW)) return 0ull;
      uint64_t v = colX[i];
      if (uint32_t(i) == (n >> 6) && (n & 63)) v &= (1ull << (n & 63)) - 1;
      return v;
    };
    for (uint32_t w = tid; w < t.Wp; w += bd) {
      const int64_t i = int64_t(w) - q;
      uint64_t v = src(i) << sh;
      if (sh) v |= src(i - 1) >> (64 - sh);
      t.M[w] = w < t.W ? v : 0ull;
    }
    if (tid == 0) {
      t.state[ST_DET_PAR] = 0;
      t.state[ST_DET_Y] = 0;
    }
  }
  __syncthreads();
  if (tid == 0) {
    t.state[ST_PIVOT] = p;
    t.kind[slot] = p != kNone ? 1 : 0;
    if (p != kNone) {
      // bytes the rowsum sweep must move: read x and z of every supported
      // column word with rows to update, write x (z) where the pivot has x (z)
      const uint64_t bytes = 8ull * s_nzw * (2ull * s_s + s_sx + s_sz);
      atomicAdd(reinterpret_cast<unsigned long long *>(t.state + ST_SWEEP_BYTES),
                (unsigned long long)bytes);
      atomicAdd(&t.state[ST_RANDOM_CNT], 1u);
    } else {
      atomicAdd(&t.state[ST_DET_CNT], 1u);
    }
  }
}

// ----------------------------------------------------------------- sweep ---
// grid = (column chunks, row-word tiles of 64); block = 4 waves; lane <-> row
// word, wave <-> every 4th column of the chunk.  Writes per-chunk counter
// partials part[chunk][w] = (c0, c1).
__device__ void det_columns(const TabDev &t, uint32_t j0, uint32_t j1, uint32_t lane, uint32_t wave) {
  uint32_t par = 0, ycnt = 0;
  for (uint32_t j = j0 + wave; j < j1; j += 4) {
    const uint64_t *cx = t.X + size_t(j) * t.Wp;
    const uint64_t *cz = t.Z + size_t(j) * t.Wp;
    uint32_t carry = 0;
    for (uint32_t wb = 0; wb < t.W; wb += 64) {
      const uint32_t w = wb + lane;
      const uint64_t T = w < t.W ? t.M[w] : 0ull;
      const uint64_t xt = T ? cx[w] & T : 0ull;
      const uint64_t zt = T ? cz[w] & T : 0ull;
      ycnt += uint32_t(__popcll(xt & zt));
      uint64_t pre = zt << 1;   // exclusive prefix parity of z inside the word
      pre ^= pre << 1; pre ^= pre << 2; pre ^= pre << 4;
      pre ^= pre << 8; pre ^= pre << 16; pre ^= pre << 32;
      const uint64_t bal = __ballot(__popcll(zt) & 1);
      const uint32_t cin = carry ^ (uint32_t(__popcll(bal & ((1ull << lane) - 1))) & 1u);
      par ^= (uint32_t(__popcll(xt & pre)) & 1u) ^ (cin & uint32_t(__popcll(xt)) & 1u);
      carry ^= uint32_t(__popcll(bal)) & 1u;
    }
  }
  const uint64_t pb = __ballot(par & 1u);
  for (int off = 32; off > 0; off >>= 1) ycnt += __shfl_xor(ycnt, off);
  if (lane == 0) {
    if (__popcll(pb) & 1) atomicXor(&t.state[ST_DET_PAR], 1u);
    if (ycnt) atomicAdd(&t.state[ST_DET_Y], ycnt);
  }
}

__global__ void __launch_bounds__(256) k_sweep(TabDev t, uint32_t a, uint32_t cols_per_chunk) {
  const uint32_t p = t.state[ST_PIVOT];
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t n = t.n;
  const uint32_t j0 = blockIdx.x * cols_per_chunk;
  const uint32_t j1 = min(n, j0 + cols_per_chunk);
  if (p == kNone) {
    if (blockIdx.y == 0) det_columns(t, j0, j1, lane, wave);
    return;
  }
  const uint32_t w = blockIdx.y * 64 + lane;
  const bool live = w < t.W;
  const uint64_t m = live ? t.M[w] : 0ull;
  const uint32_t pn = p - n, wpn = pn >> 6, wp = p >> 6;
  const uint64_t bpn = 1ull << (pn & 63), bpb = 1ull << (p & 63);
  const bool touch = live && (m != 0 || w == wpn || w == wp);
  uint64_t c0 = 0, c1 = 0;
  for (uint32_t j = j0 + wave; j < j1; j += 4) {
    const uint32_t xpj = uint32_t(t.xp[j >> 6] >> (j & 63)) & 1u;
    const uint32_t zpj = uint32_t(t.zp[j >> 6] >> (j & 63)) & 1u;
    uint64_t *px = t.X + size_t(j) * t.Wp + w;
    uint64_t *pz = t.Z + size_t(j) * t.Wp + w;
    if (!(xpj | zpj)) {
      // pivot is I here: only row p-n changes (it becomes the pivot's 0 bits)
      if (w == wpn) {
        const uint64_t x = *px, z = *pz;
        if (x & bpn) *px = x & ~bpn;
        if (z & bpn) *pz = z & ~bpn;
      }
      continue;
    }
    if (!touch) continue;
    const uint64_t x = *px, z = *pz;
    uint64_t plus, minus;
    if (xpj & zpj) {         // pivot Y: g = z - x
      plus = z & ~x;
      minus = x & ~z;
    } else if (xpj) {        // pivot X: g = z (2x - 1)
      plus = z & x;
      minus = z & ~x;
    } else {                 // pivot Z: g = x (1 - 2z)
      plus = x & ~z;
      minus = x & z;
    }
    plus &= m;
    minus &= m;
    c1 ^= c0 & plus;
    c0 ^= plus;
    c1 ^= ~c0 & minus;
    c0 ^= minus;
    uint64_t nx = xpj ? (x ^ m) : x;
    uint64_t nz = zpj ? (z ^ m) : z;
    if (w == wpn) {          // row p-n <- pivot row
      nx = xpj ? (nx | bpn) : (nx & ~bpn);
      nz = zpj ? (nz | bpn) : (nz & ~bpn);
    }
    if (w == wp) {           // row p <- Z_a
      nx &= ~bpb;
      nz = (j == a) ? (nz | bpb) : (nz & ~bpb);
    }
    if (nx != x) *px = nx;
    if (nz != z) *pz = nz;
  }
  __shared__ uint64_t s0[4][64], s1[4][64];
  s0[wave][lane] = c0;
  s1[wave][lane] = c1;
  __syncthreads();
  if (wave == 0 && live) {
#pragma unroll
    for (int k = 1; k < 4; ++k) {
      const uint64_t b0 = s0[k][lane], b1 = s1[k][lane];
      c1 ^= b1 ^ (c0 & b0);
      c0 ^= b0;
    }
    uint64_t *dst = t.part + (size_t(blockIdx.x) * t.Wp + w) * 2;
    dst[0] = c0;
    dst[1] = c1;
  }
}

// -------------------------------------------------------------- finalize ---
// grid = row-word tiles of 64; block = 16 waves.  Reduces the chunk partials,
// applies the sign update to every shot column, rewrites the signs of rows
// p-n and p, and writes the outcome.  Block 0 alone handles the
// deterministic branch.
__global__ void __launch_bounds__(1024) k_final(TabDev t, uint32_t slot, uint32_t chunks,
                                                uint64_t seed, uint64_t circuit, uint64_t shot0,
                                                uint64_t m_index) {
  const uint32_t p = t.state[ST_PIVOT];
  const uint32_t tid = threadIdx.x, lane = tid & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const uint32_t S = t.S;
  if (p == kNone) {
    if (blockIdx.x != 0) return;
    const uint32_t par = t.state[ST_DET_PAR] & 1u;
    const uint32_t y = t.state[ST_DET_Y];
    if (tid == 0 && (y & 1u)) atomicAdd(&t.state[ST_ANOMALY], 1u);
    for (uint32_t s = tid; s < S; s += blockDim.x) {
      uint32_t rt = 0;
      for (uint32_t w = 0; w < t.W; ++w) {
        const uint64_t T = t.M[w];
        if (T) rt ^= uint32_t(__popcll(T & t.R[size_t(w) * S + s])) & 1u;
      }
      t.out[size_t(slot) * S + s] = uint8_t(rt ^ par ^ ((y >> 1) & 1u));
    }
    return;
  }
  const uint32_t n = t.n;
  const uint32_t pn = p - n, wpn = pn >> 6, wp = p >> 6;
  const uint64_t bpn = 1ull << (pn & 63), bpb = 1ull << (p & 63);
  const uint32_t w = blockIdx.x * 64 + lane;
  const bool live = w < t.W;
  uint64_t c0 = 0, c1 = 0;
  if (live) {
    for (uint32_t ch = wave; ch < chunks; ch += 16) {
      const uint64_t *src = t.part + (size_t(ch) * t.Wp + w) * 2;
      const uint64_t b0 = src[0], b1 = src[1];
      c1 ^= b1 ^ (c0 & b0);
      c0 ^= b0;
    }
  }
  __shared__ uint64_t s0[16][64], s1[16][64];
  __shared__ uint64_t sM[64], sC1[64];
  s0[wave][lane] = c0;
  s1[wave][lane] = c1;
  __syncthreads();
  if (wave == 0) {
    for (int k = 1; k < 16; ++k) {
      const uint64_t b0 = s0[k][lane], b1 = s1[k][lane];
      c1 ^= b1 ^ (c0 & b0);
      c0 ^= b0;
    }
    const uint64_t mw = live ? t.M[w] : 0ull;
    uint64_t bad = c0 & mw;
    if (w == wpn) bad &= ~bpn;   // row p-n anticommutes with the pivot; overwritten below
    if (bad) atomicAdd(&t.state[ST_ANOMALY], uint32_t(__popcll(bad)));
    sM[lane] = mw;
    sC1[lane] = c1;
  }
  __syncthreads();
  const uint32_t items = 64 * S;
  for (uint32_t idx = tid; idx < items; idx += blockDim.x) {
    const uint32_t wl = idx / S, s = idx - wl * S;
    const uint32_t ww = blockIdx.x * 64 + wl;
    if (ww >= t.W) continue;
    uint64_t *pr = t.R + size_t(ww) * S + s;
    uint64_t rv = *pr;
    const uint32_t rpb = uint32_t(t.rp[s >> 6] >> (s & 63)) & 1u;
    rv ^= sM[wl] & (sC1[wl] ^ (rpb ? ~0ull : 0ull));
    if (ww == wpn) rv = rpb ? (rv | bpn) : (rv & ~bpn);
    if (ww == wp) {
      const uint32_t o = outcome_bit(seed, circuit, shot0 + s, m_index);
      rv = o ? (rv | bpb) : (rv & ~bpb);
      t.out[size_t(slot) * S + s] = uint8_t(o);
    }
    *pr = rv;
  }
}

hipError_t launch_measure_one(const TabDev &t, uint32_t a, uint32_t slot, uint64_t seed,
                              uint64_t circuit, uint64_t shot0, uint64_t m, hipStream_t st,
                              Profiler *prof) {
  const uint32_t cols = sweep_cols_per_chunk(t.n);
  const uint32_t chunks = (t.n + cols - 1) / cols;
  const uint32_t tiles = (t.W + 63) / 64;
  if (prof) prof->begin(PK_SELECT, st);
  k_select<<<1, 1024, 0, st>>>(t, a, slot);
  if (prof) prof->end(PK_SELECT, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (prof) prof->begin(PK_SWEEP, st);
  k_sweep<<<dim3(chunks, tiles), 256, 0, st>>>(t, a, cols);
  if (prof) prof->end(PK_SWEEP, st);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (prof) prof->begin(PK_FINAL, st);
  k_final<<<tiles, 1024, 0, st>>>(t, slot, chunks, seed, circuit, shot0, m);
  if (prof) prof->end(PK_FINAL, st);
  return hipGetLastError();
}

}  // namespace cliff
