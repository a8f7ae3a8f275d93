// Tableau initialisation and gate sweeps (H, S, CNOT column updates).
//
// Gate rules of the phase-space method (paper Sec. 2, after Aaronson &
// Gottesman 2004), applied to 64 rows at once with word-wise bit logic:
//   H(a):        r ^= x_a & z_a;  swap(x_a, z_a)
//   S(a):        r ^= x_a & z_a;  z_a ^= x_a
//   CNOT(a->b):  r ^= x_a & z_b & ~(x_b ^ z_a);  x_b ^= x_a;  z_a ^= z_b
// Gates on disjoint qubits touch disjoint columns and their sign terms read
// only their own columns, so every op of a layer can run concurrently; the
// sign contributions are XOR-accumulated per thread and flushed once.
#include "internal.h"

namespace cliff {

// |0...0>: X[j] has bit j (destabilizer j = X_j), Z[j] has bit n+j
// (stabilizer n+j = Z_j); signs and pending flips zero.  One pass, no memset,
// so the launch is safe inside a captured graph.
__global__ void __launch_bounds__(256) k_init_zero(TabDev t) {
  const size_t ncol = size_t(t.n) * t.Wp;
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < ncol; i += stride) {
    const uint32_t j = uint32_t(i / t.Wp), w = uint32_t(i % t.Wp);
    const uint32_t zr = t.n + j;
    t.X[i] = (w == (j >> 6)) ? (1ull << (j & 63)) : 0ull;
    t.Z[i] = (w == (zr >> 6)) ? (1ull << (zr & 63)) : 0ull;
  }
  const size_t nr = size_t(t.Wp) * t.S;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < nr; i += stride) t.R[i] = 0;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < t.Wp; i += stride) t.P[i] = 0;
}

// R[w][s] ^= P[w] for every shot (pending gate sign flips become real).
__global__ void __launch_bounds__(256) k_fold_pending(TabDev t) {
  const size_t nr = size_t(t.Wp) * t.S;
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < nr; i += stride) {
    const uint64_t p = t.P[i / t.S];
    if (p) t.R[i] ^= p;
  }
}

__global__ void __launch_bounds__(256) k_clear_pending(TabDev t) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < t.Wp; i += gridDim.x * blockDim.x)
    t.P[i] = 0;
}

__global__ void __launch_bounds__(64) k_clear_state(TabDev t) {
  if (threadIdx.x < kStateWords) t.state[threadIdx.x] = 0;
}

// One layer of ops.  Block = 4 waves; lane <-> row word (coalesced along the
// column), wave <-> a strided subset of the block's ops.
__global__ void __launch_bounds__(256) k_gate_layer(TabDev t, const uint64_t *__restrict__ ops,
                                                    uint32_t nops, uint32_t ops_per_block) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t w = blockIdx.x * 64 + lane;
  if (w >= t.W) return;
  const uint32_t o0 = blockIdx.y * ops_per_block;
  const uint32_t o1 = min(nops, o0 + ops_per_block);
  const size_t Wp = t.Wp;
  uint64_t racc = 0;
  for (uint32_t o = o0 + wave; o < o1; o += 4) {
    const uint64_t op = ops[o];
    const uint32_t a = uint32_t(op & kQubitMask);
    uint64_t *pxa = t.X + a * Wp + w;
    uint64_t *pza = t.Z + a * Wp + w;
    uint64_t xa = *pxa, za = *pza;
    if (op & OPF_HA) { racc ^= xa & za; const uint64_t tmp = xa; xa = za; za = tmp; }
    if (op & OPF_SA) { racc ^= xa & za; za ^= xa; }
    if (op & OPF_PAIR) {
      const uint32_t b = uint32_t((op >> kQubitBits) & kQubitMask);
      uint64_t *pxb = t.X + b * Wp + w;
      uint64_t *pzb = t.Z + b * Wp + w;
      uint64_t xb = *pxb, zb = *pzb;
      if (op & OPF_HB) { racc ^= xb & zb; const uint64_t tmp = xb; xb = zb; zb = tmp; }
      if (op & OPF_SB) { racc ^= xb & zb; zb ^= xb; }
      racc ^= xa & zb & ~(xb ^ za);
      xb ^= xa;
      za ^= zb;
      *pxb = xb;
      *pzb = zb;
    }
    *pxa = xa;
    *pza = za;
  }
  if (racc) atomicXor(reinterpret_cast<unsigned long long *>(t.P + w), (unsigned long long)racc);
}

// dst <- src with every sign column of dst set to src's column 0 (+ pending).
__global__ void __launch_bounds__(256) k_copy_tab(TabDev dst, TabDev src) {
  const size_t ncol = size_t(src.n) * src.Wp;
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < ncol; i += stride) {
    dst.X[i] = src.X[i];
    dst.Z[i] = src.Z[i];
  }
  const size_t nr = size_t(dst.Wp) * dst.S;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < nr; i += stride) {
    const size_t w = i / dst.S;
    dst.R[i] = src.R[w * src.S] ^ src.P[w];
  }
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < dst.Wp; i += stride) dst.P[i] = 0;
}

static inline uint32_t grid_for(size_t items, uint32_t block, uint32_t cap = 4096) {
  size_t g = (items + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return uint32_t(g);
}

hipError_t launch_init_zero(const TabDev &t, hipStream_t st) {
  const size_t items = size_t(t.n) * t.Wp;
  k_init_zero<<<grid_for(items, 256), 256, 0, st>>>(t);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_clear_state(t, st);
}

hipError_t launch_clear_state(const TabDev &t, hipStream_t st) {
  k_clear_state<<<1, 64, 0, st>>>(t);
  return hipGetLastError();
}

hipError_t launch_fold_pending(const TabDev &t, hipStream_t st) {
  k_fold_pending<<<grid_for(size_t(t.Wp) * t.S, 256), 256, 0, st>>>(t);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_clear_pending<<<grid_for(t.Wp, 256), 256, 0, st>>>(t);
  return hipGetLastError();
}

hipError_t launch_gate_layer(const TabDev &t, const uint64_t *ops, uint32_t nops, hipStream_t st) {
  if (nops == 0) return hipSuccess;
  const uint32_t tiles = (t.W + 63) / 64;
  // about 2048 blocks in total, at least 4 ops per wave
  uint32_t per = 16;
  while (size_t(tiles) * ((nops + per - 1) / per) > 2048 && per < 4096) per *= 2;
  dim3 grid(tiles, (nops + per - 1) / per);
  k_gate_layer<<<grid, 256, 0, st>>>(t, ops, nops, per);
  return hipGetLastError();
}

hipError_t launch_copy_tab(const TabDev &dst, const TabDev &src, hipStream_t st) {
  const size_t items = size_t(src.n) * src.Wp;
  k_copy_tab<<<grid_for(items, 256), 256, 0, st>>>(dst, src);
  return hipGetLastError();
}

}  // namespace cliff
