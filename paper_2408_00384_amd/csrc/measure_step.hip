// Z-measurement of a list of qubits on an HBM-resident tableau: one kernel
// launch per measurement, kernel boundaries as the only grid-wide sync.
//
// Method (paper Sec. 2, after Aaronson & Gottesman 2004): for measurement m of
// qubit a, the pivot p is the smallest stabilizer row with x_pa = 1.  If it
// exists (random outcome) every other row i with x_ia = 1 is replaced by
// row_p * row_i, the sign of the product being r_i ^ r_p ^ (sum_j g / 2 mod 2);
// row p-n takes old row p; row p becomes Z_a with a fresh random sign.  If it
// does not (deterministic outcome) the outcome is the sign of the product of
// the stabilizers n+i with x_ia = 1 and nothing changes.
//
// Work split of one step kernel (G workgroups, each owning whole columns):
//   * sweep waves: for every owned column j where the pivot is not I, every
//     64-row word with rows to update is read once and written once: the g
//     values of the 64 rows go into a bit-sliced 2-bit counter (c0, c1) per
//     row, x_j ^= M if the pivot has x_j, z_j ^= M if it has z_j, and the bits
//     of rows p-n and p are rewritten in the same pass.  One (c0, c1) pair per
//     row word and workgroup is stored as a partial.
//   * the owner of the next measured column also writes a snapshot of that
//     column and its pivot row index for the next kernel, so nobody reads a
//     column while its owner rewrites it.
//   * the last wave finishes the PREVIOUS measurement meanwhile: it reduces
//     the partials of its slice of row words across workgroups (mod 4),
//     updates the signs of every shot, rewrites the signs of rows p-n and p
//     and writes the outcome.  Signs are never read by the x/z sweep, so the
//     lag is safe; the pivot's own signs are handed on through a snapshot.
//   * deterministic outcomes are accumulated with atomics (XOR / add) and
//     assembled by a final kernel:
//       outcome = XOR_{t in T} r_t  ^  XOR_j parity(#{s<t in T: z_sj x_tj})
//                 ^ (#{(t, j): x_tj = z_tj = 1} / 2 mod 2),
//     the sign of the ordered product of rows (-1)^r i^(x.z) X^x Z^z.
#include "internal.h"
#include "philox.h"

namespace cliff {

struct StepArgs {
  uint32_t a;          // qubit measured in this step (kNone in the tail kernel)
  uint32_t a_next;     // qubit of the next step, kNone when this is the last
  uint32_t slot;       // index of this measurement within the call
  uint32_t has_prev;   // the previous measurement still needs its sign update
  uint32_t sweep;      // 0: only finish the previous measurement (tail kernel)
  uint64_t seed, circuit, shot0;
  uint64_t m_prev;     // random-bit counter index of the previous measurement
};

constexpr uint32_t kMaxOwnCols = 4096;   // columns per workgroup (pivot bits in LDS)

__device__ __forceinline__ uint64_t bit64(uint32_t b) { return 1ull << (b & 63); }

// Update mask of measurement `slot`: its column snapshot without bit p.
__device__ __forceinline__ uint64_t upd_mask(const TabDev &t, uint32_t slot, uint32_t p, uint32_t w) {
  uint64_t v = t.SN[size_t(slot % 3) * t.Wp + w];
  if (w == (p >> 6)) v &= ~bit64(p);
  return v;
}

// Product-row mask of a deterministic measurement: stabilizer rows n+i with
// x_ia = 1, i.e. the destabilizer half of the snapshot shifted up by n rows.
__device__ __forceinline__ uint64_t det_mask(const TabDev &t, uint32_t slot, uint32_t w) {
  const uint64_t *col = t.SN + size_t(slot % 3) * t.Wp;
  const uint32_t n = t.n, q = n >> 6, sh = n & 63;
  auto src = [&](int64_t i) -> uint64_t {
    if (i < 0 || i >= int64_t(t.NW)) return 0ull;
    uint64_t v = col[i];
    if (uint32_t(i) == q && sh) v &= bit64(sh) - 1;
    return v;
  };
  if (w >= t.W) return 0ull;
  const int64_t i = int64_t(w) - int64_t(q);
  uint64_t v = src(i) << sh;
  if (sh) v |= src(i - 1) >> (64 - sh);
  return v;
}

// Smallest stabilizer row set in word w of a column (for the next pivot).
__device__ __forceinline__ void note_pivot(uint32_t *s_pnext, uint32_t n, uint32_t w, uint64_t v) {
  if (w < (n >> 6)) return;
  if (w == (n >> 6)) v &= ~0ull << (n & 63);
  if (v) atomicMin(s_pnext, w * 64 + uint32_t(__builtin_ctzll(v)));
}

// Signs of the pivot row of `slot`, packed per shot, for the next kernel.
__device__ void snap_pivot_signs(const TabDev &t, uint32_t slot, uint32_t pcur, uint32_t lane) {
  const uint32_t wp = pcur >> 6, S = t.S;
  for (uint32_t sb = 0; sb < S; sb += 64) {
    const uint32_t sh = sb + lane;
    const uint32_t b = sh < S ? uint32_t(t.R[size_t(wp) * S + sh] >> (pcur & 63)) & 1u : 0u;
    const uint64_t bal = __ballot(b);
    if (lane == 0) t.rps[size_t(slot & 1) * t.SW + (sb >> 6)] = bal;
  }
}

// ---------------------------------------------- finish previous measurement
// One wave; row words w = g, g+G, ... of this workgroup.
__device__ void finish_prev(const TabDev &t, const StepArgs &s, uint32_t G, uint32_t g, uint32_t lane) {
  const uint32_t S = t.S, n = t.n;
  const uint32_t ps = s.slot - 1;
  const uint32_t pp = t.piv[ps % 4];
  const uint64_t *rps = t.rps + size_t(ps & 1) * t.SW;
  for (uint32_t w = g; w < t.W; w += G) {
    if (pp != kNone) {
      // reduce the partial counters of all workgroups for word w (mod 4)
      const uint64_t *part = t.part + size_t(ps & 1) * G * t.Wp * 2;
      uint64_t c0 = 0, c1 = 0;
      for (uint32_t q = lane; q < G; q += 64) {
        const uint64_t *src = part + (size_t(q) * t.Wp + w) * 2;
        const uint64_t b0 = src[0], b1 = src[1];
        c1 ^= b1 ^ (c0 & b0);
        c0 ^= b0;
      }
      for (int off = 32; off > 0; off >>= 1) {
        const uint64_t b0 = __shfl_xor(c0, off), b1 = __shfl_xor(c1, off);
        c1 ^= b1 ^ (c0 & b0);
        c0 ^= b0;
      }
      const uint64_t mw = upd_mask(t, ps, pp, w);
      const uint32_t ppn = pp - n;
      uint64_t bad = c0 & mw;
      if (w == (ppn >> 6)) bad &= ~bit64(ppn);   // row p-n anticommutes; overwritten below
      if (lane == 0 && bad) atomicAdd(&t.state[ST_ANOMALY], uint32_t(__popcll(bad)));
      for (uint32_t sh = lane; sh < S; sh += 64) {
        uint64_t *pr = t.R + size_t(w) * S + sh;
        uint64_t rv = *pr;
        const uint32_t rpb = uint32_t(rps[sh >> 6] >> (sh & 63)) & 1u;
        rv ^= mw & (c1 ^ (rpb ? ~0ull : 0ull));
        if (w == (ppn >> 6)) rv = rpb ? (rv | bit64(ppn)) : (rv & ~bit64(ppn));
        if (w == (pp >> 6)) {
          const uint32_t o = outcome_bit(s.seed, s.circuit, s.shot0 + sh, s.m_prev);
          rv = o ? (rv | bit64(pp)) : (rv & ~bit64(pp));
          t.out[size_t(ps) * S + sh] = uint8_t(o);
        }
        *pr = rv;
      }
    } else {
      // deterministic: XOR of the signs of the product rows in this word
      const uint64_t T = det_mask(t, ps, w);
      if (T) {
        for (uint32_t sb = 0; sb < S; sb += 64) {
          const uint32_t sh = sb + lane;
          const uint32_t par = sh < S ? uint32_t(__popcll(T & t.R[size_t(w) * S + sh])) & 1u : 0u;
          const uint64_t bal = __ballot(par);
          if (lane == 0 && bal)
            atomicXor(reinterpret_cast<unsigned long long *>(t.detr + size_t(ps) * t.SW + (sb >> 6)),
                      (unsigned long long)bal);
        }
      }
    }
  }
}

// Random-branch sweep when a wave works on one column at a time (W > 32):
// lane l holds row words K l .. K l + K - 1 of a 64 K-word tile (K = 2: one
// 16-byte access per plane), so the column and the pivot's Pauli on it are
// wave-uniform and every branch on them is scalar.  Per Pauli the g terms of
// the update rows reduce to: anti = rows anticommuting with the pivot on this
// column (pivot X: z; Z: x; Y: x ^ z), where g = +1 if (X: x; Z: ~z; Y: z)
// and -1 otherwise; adding +-1 to the 2-bit counter flips c1 where c0 equals
// that +1 condition's complement... written out:
//   X: c1 ^= anti & ~(c0 ^ x)   Z: c1 ^= anti & (c0 ^ z)   Y: c1 ^= anti & ~(c0 ^ z)
// and c0 ^= anti in every case.
template <uint32_t K>
__device__ __forceinline__ void sweep_uniform(const TabDev &t, const StepArgs &s, uint32_t p, uint32_t j0,
                                              uint32_t j1, bool own_next, uint64_t *SNn, uint32_t *s_pnext,
                                              const uint64_t *s_xp, const uint64_t *s_zp, uint64_t *s_c0,
                                              uint64_t *s_c1, uint32_t wave, uint32_t nsw, uint32_t lane,
                                              uint32_t G, uint32_t g) {
  constexpr uint32_t U = 10;   // columns in flight per lane (128 VGPRs at 1,024 threads; 12 spills)
  constexpr uint32_t Wl = 64 * K;
  const uint32_t n = t.n, W = t.W;
  const uint32_t T = (W + Wl - 1) / Wl;
  const bool whole_tiles = T >= nsw;
  const uint32_t ncg = whole_tiles ? 1u : nsw / T;
  uint32_t cgi, tfirst, tstep;
  if (whole_tiles) { cgi = 0; tfirst = wave; tstep = nsw; }
  else { cgi = wave / T; tfirst = cgi < ncg ? wave % T : T; tstep = T; }
  const uint32_t pn = p - n, wpn = pn >> 6, wp = p >> 6;
  const uint64_t bpn = bit64(pn), bpb = bit64(p);
  const uint32_t stride = T * Wl;
  for (uint32_t tile = tfirst; tile < T; tile += tstep) {
    const uint32_t w = tile * Wl + lane * K;
    const bool live = w < W;
    uint64_t m[K], c0[K], c1[K];
    bool at_pn[K], at_p[K];
    bool touch = false;
#pragma unroll
    for (uint32_t k = 0; k < K; ++k) {
      m[k] = live && w + k < W ? upd_mask(t, s.slot, p, w + k) : 0ull;
      at_pn[k] = w + k == wpn;
      at_p[k] = w + k == wp;
      touch |= m[k] != 0 || at_pn[k] || at_p[k];
      c0[k] = 0;
      c1[k] = 0;
    }
    touch &= live;
    bool has_pn = false;
#pragma unroll
    for (uint32_t k = 0; k < K; ++k) has_pn |= at_pn[k];
    for (uint32_t jb = j0 + cgi; jb < j1; jb += U * ncg) {
      uint64_t xv[U][K], zv[U][K];
      uint32_t ty[U];
      // issue the loads of U columns first ...
#pragma unroll
      for (uint32_t u = 0; u < U; ++u) {
        const uint32_t j = jb + u * ncg;
        uint32_t tj = 0;
        if (j < j1) {
          const uint32_t c = j - j0;
          tj = (uint32_t(s_xp[c >> 6] >> (c & 63)) & 1u) | ((uint32_t(s_zp[c >> 6] >> (c & 63)) & 1u) << 1);
        }
        tj = __builtin_amdgcn_readfirstlane(tj);
        ty[u] = tj;
        const bool nxt = own_next && j == s.a_next;
        // supported column: every word with rows to update; pivot I here:
        // only the word of row p-n (it becomes the pivot's zeros)
        const bool need = j < j1 && live && (nxt || (tj ? touch : has_pn));
        const size_t at = size_t(j) * t.Wp + w;
        if constexpr (K == 2) {
          ulonglong2 vx = make_ulonglong2(0, 0), vz = make_ulonglong2(0, 0);
          if (need) {
            vx = *reinterpret_cast<const ulonglong2 *>(t.X + at);
            vz = *reinterpret_cast<const ulonglong2 *>(t.Z + at);
          }
          xv[u][0] = vx.x; xv[u][1] = vx.y;
          zv[u][0] = vz.x; zv[u][1] = vz.y;
        } else {
          xv[u][0] = need ? t.X[at] : 0ull;
          zv[u][0] = need ? t.Z[at] : 0ull;
        }
      }
      // ... then update them
#pragma unroll
      for (uint32_t u = 0; u < U; ++u) {
        const uint32_t j = jb + u * ncg;
        if (j >= j1) continue;   // uniform
        const uint32_t tj = ty[u];
        const bool nxt = own_next && j == s.a_next;
        if (!live || !(nxt || (tj ? touch : has_pn))) continue;
        uint64_t nx[K], nz[K];
        bool chx = false, chz = false;
#pragma unroll
        for (uint32_t k = 0; k < K; ++k) {
          const uint64_t x = xv[u][k], z = zv[u][k];
          uint64_t ax = x, az = z;
          if (tj == 1u) {          // pivot X on this column
            const uint64_t anti = z & m[k];
            c1[k] ^= anti & ~(c0[k] ^ x);
            c0[k] ^= anti;
            ax = x ^ m[k];
          } else if (tj == 2u) {   // pivot Z
            const uint64_t anti = x & m[k];
            c1[k] ^= anti & (c0[k] ^ z);
            c0[k] ^= anti;
            az = z ^ m[k];
          } else if (tj == 3u) {   // pivot Y
            const uint64_t anti = (x ^ z) & m[k];
            c1[k] ^= anti & ~(c0[k] ^ z);
            c0[k] ^= anti;
            ax = x ^ m[k];
            az = z ^ m[k];
          }
          if (at_pn[k]) {   // row p-n <- pivot row
            ax = (tj & 1u) ? (ax | bpn) : (ax & ~bpn);
            az = (tj & 2u) ? (az | bpn) : (az & ~bpn);
          }
          if (at_p[k]) {    // row p <- Z_a
            ax &= ~bpb;
            az = (j == s.a) ? (az | bpb) : (az & ~bpb);
          }
          nx[k] = ax;
          nz[k] = az;
          chx |= ax != x;
          chz |= az != z;
        }
        const size_t at = size_t(j) * t.Wp + w;
        if constexpr (K == 2) {
          if (chx) *reinterpret_cast<ulonglong2 *>(t.X + at) = make_ulonglong2(nx[0], nx[1]);
          if (chz) *reinterpret_cast<ulonglong2 *>(t.Z + at) = make_ulonglong2(nz[0], nz[1]);
        } else {
          if (chx) t.X[at] = nx[0];
          if (chz) t.Z[at] = nz[0];
        }
        if (nxt) {
#pragma unroll
          for (uint32_t k = 0; k < K; ++k)
            if (w + k < W) {
              SNn[w + k] = nx[k];
              note_pivot(s_pnext, n, w + k, nx[k]);
            }
        }
      }
    }
    if (whole_tiles) {
      if (live) {   // complete over the workgroup's columns: store directly
        uint64_t *part = t.part + (size_t(s.slot & 1) * G + g) * t.Wp * 2;
#pragma unroll
        for (uint32_t k = 0; k < K; ++k) {
          part[size_t(w + k) * 2] = c0[k];
          part[size_t(w + k) * 2 + 1] = c1[k];
        }
      }
    } else if (cgi < ncg) {
#pragma unroll
      for (uint32_t k = 0; k < K; ++k) {
        s_c0[cgi * stride + w + k] = c0[k];
        s_c1[cgi * stride + w + k] = c1[k];
      }
    }
  }
}

// ------------------------------------------------------------------ step ---
__global__ void __launch_bounds__(1024) k_step(TabDev t, StepArgs s) {
  __shared__ uint64_t s_c0[2048], s_c1[2048];
  __shared__ uint64_t s_xp[kMaxOwnCols / 64], s_zp[kMaxOwnCols / 64];
  __shared__ uint32_t s_pnext;
  const uint32_t tid = threadIdx.x, lane = tid & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const uint32_t nw = blockDim.x >> 6;   // >= 2
  const uint32_t G = gridDim.x, g = blockIdx.x;
  const uint32_t n = t.n, W = t.W;

  if (!s.sweep) {   // tail: finish the last measurement of the call
    if (wave == 0 && s.has_prev) finish_prev(t, s, G, g, lane);
    return;
  }
  if (tid == 0) s_pnext = kNone;
  const uint32_t rwave = nw - 1;         // finishes the previous measurement
  const uint32_t nsw = nw - 1;           // sweep waves
  const uint32_t p = t.piv[s.slot % 4];
  if (g == 0 && tid == 0) t.kind[s.slot] = p != kNone ? 1 : 0;
  const uint32_t j0 = uint32_t(uint64_t(g) * n / G), j1 = uint32_t(uint64_t(g + 1) * n / G);
  const bool own_next = s.a_next != kNone && s.a_next >= j0 && s.a_next < j1;
  uint64_t *SNn = t.SN + size_t((s.slot + 1) % 3) * t.Wp;
  if (p != kNone) {
    // pivot row bits of the owned columns, read before any wave rewrites the
    // word that holds row p
    const uint32_t wp = p >> 6, C = j1 - j0;
    for (uint32_t c = tid; c < ((C + 63) & ~63u); c += blockDim.x) {
      uint32_t xb = 0, zb = 0;
      if (c < C) {
        xb = uint32_t(t.X[size_t(j0 + c) * t.Wp + wp] >> (p & 63)) & 1u;
        zb = uint32_t(t.Z[size_t(j0 + c) * t.Wp + wp] >> (p & 63)) & 1u;
      }
      const uint64_t bx = __ballot(xb), bz = __ballot(zb);
      if (lane == 0) { s_xp[c >> 6] = bx; s_zp[c >> 6] = bz; }
    }
  }
  __syncthreads();

  if (wave == rwave) {
    if (s.has_prev) finish_prev(t, s, G, g, lane);
    if (p != kNone && ((p >> 6) % G) == g) snap_pivot_signs(t, s.slot, p, lane);
  }

  // lane layout: Wl words per column segment, cpw column segments per wave
  // (W > 32: one column per wave, K = 2 words per lane from W = 128 on)
  const bool uniform = W > 32;
  const uint32_t Wl = W >= 128 ? 128u : W > 32 ? 64u : (W <= 1 ? 1u : (1u << (32 - __builtin_clz(W - 1))));
  const uint32_t cpw = uniform ? 1u : 64 / Wl;
  const uint32_t T = (W + Wl - 1) / Wl;             // word tiles
  const bool whole_tiles = T >= nsw;                 // each wave owns whole tiles
  const uint32_t ncg = whole_tiles ? 1u : nsw / T;   // column groups per tile
  const uint32_t sub = lane / Wl, wl = lane % Wl;
  const uint32_t stride = T * Wl;                    // LDS row of one column slot

  if (p != kNone && wave != rwave && uniform) {
    if (W >= 128)
      sweep_uniform<2>(t, s, p, j0, j1, own_next, SNn, &s_pnext, s_xp, s_zp, s_c0, s_c1, wave, nsw, lane, G, g);
    else
      sweep_uniform<1>(t, s, p, j0, j1, own_next, SNn, &s_pnext, s_xp, s_zp, s_c0, s_c1, wave, nsw, lane, G, g);
  } else if (p != kNone && wave != rwave) {
    // ------------------------------------------- random branch, W <= 32
    const uint32_t pn = p - n, wpn = pn >> 6, wp = p >> 6;
    const uint64_t bpn = bit64(pn), bpb = bit64(p);
    uint32_t cgi, tfirst, tstep;
    if (whole_tiles) { cgi = 0; tfirst = wave; tstep = nsw; }
    else { cgi = wave / T; tfirst = cgi < ncg ? wave % T : T; tstep = T; }
    const uint32_t cslot = cgi * cpw + sub, cstride = ncg * cpw;
    constexpr uint32_t U = 8;   // columns in flight per lane
    for (uint32_t tile = tfirst; tile < T; tile += tstep) {
      const uint32_t w = tile * Wl + wl;
      const bool live = w < W;
      const uint64_t m = live ? upd_mask(t, s.slot, p, w) : 0ull;
      const bool touch = live && (m != 0 || w == wpn || w == wp);
      uint64_t c0 = 0, c1 = 0;
      for (uint32_t jb = j0 + cslot; jb < j1; jb += U * cstride) {
        uint64_t xv[U], zv[U];
        uint32_t ty[U];
        bool need[U];
        // issue the loads of U columns first ...
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
          const uint32_t j = jb + u * cstride;
          uint32_t tj = 0;
          if (j < j1) {
            const uint32_t c = j - j0;
            tj = (uint32_t(s_xp[c >> 6] >> (c & 63)) & 1u) | ((uint32_t(s_zp[c >> 6] >> (c & 63)) & 1u) << 1);
          }
          const bool nxt = own_next && j == s.a_next;
          // supported column: every word with rows to update; pivot I here:
          // only the word of row p-n (it becomes the pivot's zeros)
          need[u] = j < j1 && live && (nxt || (tj ? touch : (w == wpn)));
          ty[u] = tj;
          xv[u] = need[u] ? t.X[size_t(j) * t.Wp + w] : 0ull;
          zv[u] = need[u] ? t.Z[size_t(j) * t.Wp + w] : 0ull;
        }
        // ... then update them
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
          if (!need[u]) continue;
          const uint32_t j = jb + u * cstride;
          const uint64_t x = xv[u], z = zv[u];
          const uint64_t X1 = (ty[u] & 1u) ? ~0ull : 0ull, Z1 = (ty[u] & 2u) ? ~0ull : 0ull;
          const uint64_t yc = X1 & Z1, xc = X1 & ~Z1, zc = ~X1 & Z1;
          // g = +1 / -1 per row: pivot Y: z-x;  pivot X: z(2x-1);  pivot Z: x(1-2z)
          const uint64_t plus = ((yc & z & ~x) | (xc & z & x) | (zc & x & ~z)) & m;
          const uint64_t minus = ((yc & x & ~z) | (xc & z & ~x) | (zc & x & z)) & m;
          c1 ^= c0 & plus;
          c0 ^= plus;
          c1 ^= ~c0 & minus;
          c0 ^= minus;
          uint64_t nx = x ^ (X1 & m), nz = z ^ (Z1 & m);
          if (w == wpn) {   // row p-n <- pivot row
            nx = (ty[u] & 1u) ? (nx | bpn) : (nx & ~bpn);
            nz = (ty[u] & 2u) ? (nz | bpn) : (nz & ~bpn);
          }
          if (w == wp) {    // row p <- Z_a
            nx &= ~bpb;
            nz = (j == s.a) ? (nz | bpb) : (nz & ~bpb);
          }
          if (nx != x) t.X[size_t(j) * t.Wp + w] = nx;
          if (nz != z) t.Z[size_t(j) * t.Wp + w] = nz;
          if (own_next && j == s.a_next) {
            SNn[w] = nx;
            note_pivot(&s_pnext, n, w, nx);
          }
        }
      }
      if (whole_tiles) {
        if (live) {   // complete over the workgroup's columns: store directly
          uint64_t *part = t.part + (size_t(s.slot & 1) * G + g) * t.Wp * 2;
          part[size_t(w) * 2] = c0;
          part[size_t(w) * 2 + 1] = c1;
        }
      } else if (cgi < ncg) {
        s_c0[cslot * stride + tile * Wl + wl] = c0;
        s_c1[cslot * stride + tile * Wl + wl] = c1;
      }
    }
  } else if (p == kNone && wave != rwave) {
    // -------------------------------------------------- deterministic branch
    uint32_t par = 0, ycnt = 0;
    for (uint32_t j = j0 + wave; j < j1; j += nsw) {
      const uint64_t *cx = t.X + size_t(j) * t.Wp;
      const uint64_t *cz = t.Z + size_t(j) * t.Wp;
      uint32_t carry = 0;
      for (uint32_t wb = 0; wb < W; wb += 64) {
        const uint32_t w = wb + lane;
        const uint64_t Tm = det_mask(t, s.slot, w);
        const uint64_t xt = Tm ? cx[w] & Tm : 0ull;
        const uint64_t zt = Tm ? cz[w] & Tm : 0ull;
        ycnt += uint32_t(__popcll(xt & zt));
        uint64_t pre = zt << 1;   // exclusive prefix parity of z inside the word
        pre ^= pre << 1; pre ^= pre << 2; pre ^= pre << 4;
        pre ^= pre << 8; pre ^= pre << 16; pre ^= pre << 32;
        const uint64_t bal = __ballot(__popcll(zt) & 1);
        const uint32_t cin = carry ^ (uint32_t(__popcll(bal & (bit64(lane) - 1))) & 1u);
        par ^= (uint32_t(__popcll(xt & pre)) & 1u) ^ (cin & uint32_t(__popcll(xt)) & 1u);
        carry ^= uint32_t(__popcll(bal)) & 1u;
      }
    }
    const uint64_t pb = __ballot(par & 1u);
    for (int off = 32; off > 0; off >>= 1) ycnt += __shfl_xor(ycnt, off);
    if (lane == 0) {
      if (__popcll(pb) & 1) atomicXor(&t.detpar[s.slot], 1u);
      if (ycnt) atomicAdd(&t.detY[s.slot], ycnt);
    }
    if (own_next) {   // the next column is unchanged: copy it to the snapshot
      const uint64_t *cx = t.X + size_t(s.a_next) * t.Wp;
      for (uint32_t w = wave * 64 + lane; w < W; w += nsw * 64) {
        const uint64_t x = cx[w];
        SNn[w] = x;
        note_pivot(&s_pnext, n, w, x);
      }
    }
  }
  __syncthreads();
  if (p != kNone && !whole_tiles) {
    // combine the column slots of every word into the workgroup partial
    const uint32_t slots = ncg * cpw;
    uint64_t *part = t.part + (size_t(s.slot & 1) * G + g) * t.Wp * 2;
    for (uint32_t w = tid; w < W; w += blockDim.x) {
      uint64_t c0 = 0, c1 = 0;
      for (uint32_t cs = 0; cs < slots; ++cs) {
        const uint64_t b0 = s_c0[cs * stride + w], b1 = s_c1[cs * stride + w];
        c1 ^= b1 ^ (c0 & b0);
        c0 ^= b0;
      }
      part[size_t(w) * 2] = c0;
      part[size_t(w) * 2 + 1] = c1;
    }
  }
  if (tid == 0 && own_next) t.piv[(s.slot + 1) % 4] = s_pnext;
  if (tid == 0) {
    if (p != kNone) {
      // this workgroup's columns' share of 2 s + s_x + s_z (pivot-row support)
      uint32_t sx = 0, sz = 0, sxz = 0;
      for (uint32_t k = 0; k < (j1 - j0 + 63) / 64; ++k) {
        sx += uint32_t(__popcll(s_xp[k]));
        sz += uint32_t(__popcll(s_zp[k]));
        sxz += uint32_t(__popcll(s_xp[k] | s_zp[k]));
      }
      const uint64_t sup = 2ull * sxz + sx + sz;
      if (sup)
        atomicAdd(reinterpret_cast<unsigned long long *>(t.state + ST_SUPPORT),
                  (unsigned long long)sup);
    }
    if (g == 0) atomicAdd(&t.state[p != kNone ? ST_RANDOM_CNT : ST_DET_CNT], 1u);
  }
}

// ---------------------------------------------------------- call prologue ---
// Snapshot of the first measured column, its pivot, and cleared accumulators.
__global__ void __launch_bounds__(1024) k_begin(TabDev t, uint32_t a0, uint32_t k) {
  __shared__ uint32_t s_p;
  const uint32_t tid = threadIdx.x;
  if (tid == 0) s_p = kNone;
  __syncthreads();
  const uint64_t *col = t.X + size_t(a0) * t.Wp;
  for (uint32_t w = tid; w < t.Wp; w += blockDim.x) {
    const uint64_t x = w < t.W ? col[w] : 0ull;
    t.SN[w] = x;
    note_pivot(&s_p, t.n, w, x);
  }
  for (uint32_t i = tid; i < k; i += blockDim.x) {
    t.detpar[i] = 0;
    t.detY[i] = 0;
  }
  for (size_t i = tid; i < size_t(k) * t.SW; i += blockDim.x) t.detr[i] = 0;
  __syncthreads();
  if (tid == 0) t.piv[0] = s_p;
}

// ------------------------------------------------------- call epilogue ---
// Outcomes of the deterministic measurements from the accumulated terms.
__global__ void __launch_bounds__(256) k_det_out(TabDev t, uint32_t k) {
  const uint32_t S = t.S;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < size_t(k) * S;
       i += size_t(gridDim.x) * blockDim.x) {
    const uint32_t slot = uint32_t(i / S), sh = uint32_t(i % S);
    if (t.kind[slot]) continue;
    const uint32_t y = t.detY[slot];
    if (sh == 0 && (y & 1u)) atomicAdd(&t.state[ST_ANOMALY], 1u);
    const uint32_t r = uint32_t(t.detr[size_t(slot) * t.SW + (sh >> 6)] >> (sh & 63)) & 1u;
    t.out[i] = uint8_t(r ^ (t.detpar[slot] & 1u) ^ ((y >> 1) & 1u));
  }
}

hipError_t launch_measure_list(const TabDev &t, const uint32_t *qubits, uint32_t k, uint64_t seed,
                               uint64_t circuit, uint64_t shot0, uint64_t m0, hipStream_t st,
                               Profiler *prof) {
  if (k == 0) return hipSuccess;
  const uint32_t G = step_grid(t.n), B = step_block(t.n);
  if (prof) prof->begin(PK_SELECT, st);
  k_begin<<<1, 1024, 0, st>>>(t, qubits[0], k);
  if (prof) prof->end(PK_SELECT, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (uint32_t i = 0; i <= k; ++i) {
    StepArgs a;
    a.slot = i;
    a.sweep = i < k ? 1u : 0u;
    a.a = i < k ? qubits[i] : kNone;
    a.a_next = i + 1 < k ? qubits[i + 1] : kNone;
    a.has_prev = i > 0 ? 1u : 0u;
    a.seed = seed;
    a.circuit = circuit;
    a.shot0 = shot0;
    a.m_prev = m0 + i - 1;
    if (prof) prof->begin(a.sweep ? PK_SWEEP : PK_FINAL, st);
    k_step<<<G, a.sweep ? B : 64 * 2, 0, st>>>(t, a);
    if (prof) prof->end(a.sweep ? PK_SWEEP : PK_FINAL, st);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (prof) prof->begin(PK_FINAL, st);
  k_det_out<<<(k * t.S + 255) / 256 < 1024 ? (k * t.S + 255) / 256 : 1024, 256, 0, st>>>(t, k);
  if (prof) prof->end(PK_FINAL, st);
  return hipGetLastError();
}

}  // namespace cliff
