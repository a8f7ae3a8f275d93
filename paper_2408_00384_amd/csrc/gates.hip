// Tableau initialisation and gate sweeps (column updates).
//
// Gate rules of the phase-space method (paper Sec. 2, after Aaronson &
// Gottesman 2004), applied to 64 rows at once with word-wise bit logic:
//   H(a):        r ^= x_a & z_a;  swap(x_a, z_a)
//   S(a):        r ^= x_a & z_a;  z_a ^= x_a
//   CNOT(a->b):  r ^= x_a & z_b & ~(x_b ^ z_a);  x_b ^= x_a;  z_a ^= z_b
// and the rest of the Clifford gate set (S^dagger, X, Y, Z, CZ, SWAP) in the
// same form; an op word carries one single-qubit Clifford per qubit and one
// two-qubit gate (the encoding and rules are in gate_ops.h).
// Gates on disjoint qubits touch disjoint columns and their sign terms read
// only their own columns, so every op of a layer can run concurrently; the
// sign contributions are XOR-accumulated per thread and flushed once.
#include <string.h>

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
  if (blockIdx.x == 0 && threadIdx.x == 0) *t.abort_flag = 0;
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
    if (!op_valid(op, t.n)) continue;   // malformed op
    const uint32_t a = op_a(op), pair = op_pair(op);
    uint64_t *pxa = t.X + a * Wp + w;
    uint64_t *pza = t.Z + a * Wp + w;
    uint64_t xa = *pxa, za = *pza;
    if (op_ca(op)) sq_apply(op_ca(op), xa, za, racc);
    if (pair != PAIR_NONE) {
      const uint32_t b = op_b(op);
      uint64_t *pxb = t.X + b * Wp + w;
      uint64_t *pzb = t.Z + b * Wp + w;
      uint64_t xb = *pxb, zb = *pzb;
      if (op_cb(op)) sq_apply(op_cb(op), xb, zb, racc);
      pair_apply(pair, xa, za, xb, zb, racc);
      *pxb = xb;
      *pzb = zb;
    }
    *pxa = xa;
    *pza = za;
  }
  if (racc) atomicXor(reinterpret_cast<unsigned long long *>(t.P + w), (unsigned long long)racc);
}

typedef __attribute__((address_space(1))) const uint64_t GlobalU64;
typedef __attribute__((address_space(1))) const uint32_t GlobalU32;

__device__ __forceinline__ void lds_xor(uint32_t *p, uint32_t v) { atomicXor(p, v); }
__device__ __forceinline__ void lds_xor(uint64_t *p, uint64_t v) {
  atomicXor(reinterpret_cast<unsigned long long *>(p), (unsigned long long)v);
}
__device__ __forceinline__ void lds_xor(U128 *p, U128 v) {
  lds_xor(&p->lo, v.lo);
  lds_xor(&p->hi, v.hi);
}
__device__ __forceinline__ bool nonzero(uint32_t v) { return v != 0; }
__device__ __forceinline__ bool nonzero(uint64_t v) { return v != 0; }
__device__ __forceinline__ bool nonzero(U128 v) { return (v.lo | v.hi) != 0; }

// All layers of a gate stream in one launch.  Gates act row by row, so a
// workgroup that owns a group of rows (32 or 64: the bits of T) of every
// column can apply every layer to them without talking to any other
// workgroup: it loads its row group of X and Z into LDS (2 n sizeof(T)
// bytes), runs the layers with a workgroup barrier between consecutive
// layers, and writes them back once.  Its sign flips stay in registers and
// land in its own part of P.
template <typename T>
__device__ __forceinline__ void apply_op_lds(uint64_t op, uint32_t n, T *sx, T *sz, T &racc) {
  if (!op_valid(op, n)) return;   // malformed op
  const uint32_t a = op_a(op), pair = op_pair(op);
  T xa = sx[a], za = sz[a];
  if (op_ca(op)) sq_apply(op_ca(op), xa, za, racc);
  if (pair != PAIR_NONE) {
    const uint32_t b = op_b(op);
    T xb = sx[b], zb = sz[b];
    if (op_cb(op)) sq_apply(op_cb(op), xb, zb, racc);
    pair_apply(pair, xa, za, xb, zb, racc);
    sx[b] = xb;
    sz[b] = zb;
  }
  sx[a] = xa;
  sz[a] = za;
}

template <typename T>
__device__ __forceinline__ void fused_body(uint64_t *X, uint64_t *Z, uint64_t *P, uint32_t n, uint32_t Wp,
                                           const uint64_t *__restrict__ ops,
                                           const uint32_t *__restrict__ offs, uint32_t depth,
                                           uint32_t unit, T *sx, T *sz, T *s_r) {
  const uint32_t tid = threadIdx.x, lane = tid & 63, nthr = blockDim.x;
  const size_t cs = size_t(Wp) * 8 / sizeof(T);  // column stride in T words (Wp is a multiple of 8)
  const T *XT = reinterpret_cast<const T *>(X);
  const T *ZT = reinterpret_cast<const T *>(Z);
  for (uint32_t j = tid; j < n; j += nthr) {
    sx[j] = XT[j * cs + unit];
    sz[j] = ZT[j * cs + unit];
  }
  if (tid == 0) *s_r = T{};
  __syncthreads();
  // The op stream and the offsets are read through global-address-space
  // pointers: global (not flat) loads count only in vmcnt, so the LDS waits
  // of a layer do not wait for them.
  const GlobalU64 *gops = (const GlobalU64 *)ops;
  const GlobalU32 *goffs = (const GlobalU32 *)offs;
  // Layer boundaries: lane i of every wave holds offs[base + i] of the
  // current block of 64 (one load per 64 layers); a layer reads its two
  // bounds with readlane.  The first op of the next layer is loaded while
  // the current layer runs, so its latency hides behind the LDS work.
  uint32_t base = 0, offv = lane <= depth ? goffs[lane] : 0u;
  auto bound = [&](uint32_t i) -> uint32_t {   // offs[i], i uniform, i <= depth
    if ((i & ~63u) != base) {
      base = i & ~63u;
      offv = base + lane <= depth ? goffs[base + lane] : 0u;
    }
    return uint32_t(__builtin_amdgcn_readlane(int(offv), int(i & 63u)));
  };
  T racc{};
  uint32_t lo = bound(0), hi = depth ? bound(1) : lo;
  uint64_t nxt = lo + tid < hi ? gops[lo + tid] : 0ull;
  for (uint32_t l = 0; l < depth; ++l) {
    const uint32_t a0 = lo, a1 = hi;
    const uint64_t cur = nxt;
    if (l + 1 < depth) {
      lo = a1;
      hi = bound(l + 2);
      nxt = lo + tid < hi ? gops[lo + tid] : 0ull;
    }
    if (a0 + tid < a1) apply_op_lds(cur, n, sx, sz, racc);
    for (uint32_t k = a0 + tid + nthr; k < a1; k += nthr) apply_op_lds(uint64_t(gops[k]), n, sx, sz, racc);
    lds_barrier();
  }
  if (nonzero(racc)) lds_xor(s_r, racc);
  T *XW = reinterpret_cast<T *>(X);
  T *ZW = reinterpret_cast<T *>(Z);
  for (uint32_t j = tid; j < n; j += nthr) {
    XW[j * cs + unit] = sx[j];
    ZW[j * cs + unit] = sz[j];
  }
  __syncthreads();
  if (tid == 0 && nonzero(*s_r)) reinterpret_cast<T *>(P)[unit] ^= *s_r;   // this part of P is ours alone
}

// One tableau, 32-row groups (twice as many workgroups as 64-row ones: a
// single tableau is latency-bound, not throughput-bound).  Launched with up
// to 1024 threads: 16 waves share a group's layer work, so that more LDS
// round trips are in flight per SIMD (n = 10,000, 20 layers: 30 % less time
// than with 256 threads).
constexpr uint32_t kFusedMaxThreads = 1024;
__global__ void __launch_bounds__(kFusedMaxThreads) k_gates_fused(TabDev t, const uint64_t *__restrict__ ops,
                                                     const uint32_t *__restrict__ offs, uint32_t depth) {
  extern __shared__ uint64_t lds_u64[];
  __shared__ uint32_t s_r;
  uint32_t *sx = reinterpret_cast<uint32_t *>(lds_u64), *sz = sx + t.n;
  fused_body<uint32_t>(t.X, t.Z, t.P, t.n, t.Wp, ops, offs, depth, blockIdx.x, sx, sz, &s_r);
}

// Many tableaux in one launch: blockIdx.y picks the tableau, blockIdx.x its
// row group (groups past the tableau's 2n rows exit at once).
template <typename T>
__global__ void __launch_bounds__(256) k_gates_many(const ManyDesc *__restrict__ descs) {
  extern __shared__ uint64_t lds_u64[];
  __shared__ T s_r;
  const ManyDesc d = descs[blockIdx.y];
  constexpr uint32_t kBits = 8 * sizeof(T);
  if (blockIdx.x >= (2 * d.n + kBits - 1) / kBits) return;   // group past the tableau's 2n rows
  T *sx = reinterpret_cast<T *>(lds_u64), *sz = sx + d.n;
  fused_body<T>(d.X, d.Z, d.P, d.n, d.Wp, d.ops, d.offs, d.depth, blockIdx.x, sx, sz, &s_r);
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
  if (blockIdx.x == 0 && threadIdx.x == 0) *dst.abort_flag = 0;
}

// Words handed over in the kernel's arguments, stored to device memory (an
// upload that needs no staging buffer and no host-memory copy).
constexpr uint32_t kArgWords = 960;
struct ArgWords {
  uint32_t w[kArgWords];
};
__global__ void __launch_bounds__(256) k_store_words(uint32_t *dst, ArgWords a, uint32_t count) {
  for (uint32_t i = threadIdx.x; i < count; i += blockDim.x) dst[i] = a.w[i];
}

// Word words[q] of every column of X and Z, gathered for a host readout of a
// few rows: ox[q * n + j] = X[j * Wp + words[q]] (every words[q] < W).
__global__ void __launch_bounds__(256) k_gather_words(TabDev t, const uint32_t *__restrict__ words, uint32_t nw,
                                                      uint64_t *__restrict__ ox, uint64_t *__restrict__ oz) {
  const size_t total = size_t(nw) * t.n;
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += stride) {
    const size_t q = i / t.n, j = i % t.n;
    const size_t at = j * t.Wp + words[q];
    ox[i] = t.X[at];
    oz[i] = t.Z[at];
  }
}

// Outcomes of the last measurement pass (staging: out[i * S + s], kind[i])
// into a caller's record: rec[s * ld + col0 + i], random flags rnd[col0 + i].
__global__ void __launch_bounds__(256) k_record(TabDev t, uint32_t cnt, uint8_t *__restrict__ rec, size_t ld,
                                                size_t col0, uint8_t *__restrict__ rnd) {
  const size_t total = size_t(cnt) * t.S;
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t j = size_t(blockIdx.x) * blockDim.x + threadIdx.x; j < total; j += stride) {
    const size_t s = j / cnt, i = j % cnt;
    rec[s * ld + col0 + i] = t.out[i * t.S + s];
  }
  if (rnd)
    for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < cnt; i += stride) rnd[col0 + i] = t.kind[i];
}

// Classically conditioned Paulis: op i = qubit (bits 0..23) | Pauli (bits
// 24..25: 1 X, 2 Y, 3 Z) | record column (bits 32..63).  In shot s, when
// rec[s * ld + column] is 1, every row that anticommutes with the Pauli
// flips sign: X flips rows with z_a = 1, Z rows with x_a = 1, Y rows with
// x_a ^ z_a = 1.  Thread <-> (row word, shot); the ops only XOR into signs,
// so their order does not matter.
__global__ void __launch_bounds__(256) k_cond_pauli(TabDev t, const uint64_t *__restrict__ ops, uint32_t k,
                                                    const uint8_t *__restrict__ rec, size_t ld) {
  const size_t total = size_t(t.W) * t.S;
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t j = size_t(blockIdx.x) * blockDim.x + threadIdx.x; j < total; j += stride) {
    const size_t w = j / t.S, s = j % t.S;
    uint64_t flip = 0;
    for (uint32_t i = 0; i < k; ++i) {
      const uint64_t op = ops[i];
      const uint32_t a = uint32_t(op & kQubitMask), p = uint32_t(op >> 24) & 3u;
      if (a >= t.n || !(rec[s * ld + (op >> 32)] & 1u)) continue;
      const uint64_t x = t.X[size_t(a) * t.Wp + w], z = t.Z[size_t(a) * t.Wp + w];
      // the Pauli's x part (X, Y) flips rows with z = 1, its z part (Y, Z) rows with x = 1
      flip ^= (p != 3u ? z : 0ull) ^ (p != 1u ? x : 0ull);
    }
    if (flip) t.R[w * t.S + s] ^= flip;
  }
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

bool fused_gates_fit(uint32_t n) { return size_t(n) * 8 <= kFusedGateLds; }

hipError_t launch_gates_fused(const TabDev &t, const uint64_t *ops, const uint32_t *dev_offs,
                              uint32_t depth, hipStream_t st) {
  if (depth == 0) return hipSuccess;
  const size_t lds = size_t(t.n) * 8;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_gates_fused),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(kFusedGateLds));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  const uint32_t halves = (2 * t.n + 31) / 32;
  // (below n = 512 a layer has too few ops for 16 waves)
  const uint32_t threads = t.n >= 512 ? kFusedMaxThreads : 256;
  k_gates_fused<<<halves, threads, lds, st>>>(t, ops, dev_offs, depth);
  return hipGetLastError();
}

bool many_gates_fit(uint32_t max_n, uint32_t rows) { return 2 * size_t(max_n) * (rows / 8) <= kFusedGateLds; }

hipError_t launch_gates_many(const ManyDesc *dev_descs, uint32_t count, uint32_t max_n, uint32_t rows,
                             hipStream_t st) {
  if (count == 0) return hipSuccess;
  const int v = rows == 128 ? 2 : rows == 64 ? 1 : 0;
  const void *fn = v == 2 ? reinterpret_cast<const void *>(k_gates_many<U128>)
                 : v == 1 ? reinterpret_cast<const void *>(k_gates_many<uint64_t>)
                          : reinterpret_cast<const void *>(k_gates_many<uint32_t>);
  static bool attr_set[3] = {false, false, false};
  if (!attr_set[v]) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(kFusedGateLds));
    if (e != hipSuccess) return e;
    attr_set[v] = true;
  }
  const size_t lds = 2 * size_t(max_n) * (rows / 8);
  const dim3 grid((2 * max_n + rows - 1) / rows, count);
  if (v == 2)
    k_gates_many<U128><<<grid, 256, lds, st>>>(dev_descs);
  else if (v == 1)
    k_gates_many<uint64_t><<<grid, 256, lds, st>>>(dev_descs);
  else
    k_gates_many<uint32_t><<<grid, 256, lds, st>>>(dev_descs);
  return hipGetLastError();
}

hipError_t launch_record(const TabDev &t, uint32_t cnt, uint8_t *rec, size_t ld, size_t col0, uint8_t *rnd,
                         hipStream_t st) {
  if (cnt == 0) return hipSuccess;
  k_record<<<grid_for(size_t(cnt) * t.S, 256), 256, 0, st>>>(t, cnt, rec, ld, col0, rnd);
  return hipGetLastError();
}

hipError_t launch_cond_pauli(const TabDev &t, const uint64_t *ops, uint32_t k, const uint8_t *rec, size_t ld,
                             hipStream_t st) {
  if (k == 0) return hipSuccess;
  k_cond_pauli<<<grid_for(size_t(t.W) * t.S, 256), 256, 0, st>>>(t, ops, k, rec, ld);
  return hipGetLastError();
}

hipError_t launch_gather_words(const TabDev &t, const uint32_t *words, uint32_t nw, uint64_t *ox, uint64_t *oz,
                               hipStream_t st) {
  if (nw == 0) return hipSuccess;
  k_gather_words<<<grid_for(size_t(nw) * t.n, 256), 256, 0, st>>>(t, words, nw, ox, oz);
  return hipGetLastError();
}

hipError_t launch_copy_tab(const TabDev &dst, const TabDev &src, hipStream_t st) {
  const size_t items = size_t(src.n) * src.Wp;
  k_copy_tab<<<grid_for(items, 256), 256, 0, st>>>(dst, src);
  return hipGetLastError();
}

hipError_t launch_store_words(uint32_t *dst, const uint32_t *host, uint32_t count, hipStream_t st) {
  for (uint32_t at = 0; at < count; at += kArgWords) {
    ArgWords a;
    const uint32_t c = count - at < kArgWords ? count - at : kArgWords;
    memcpy(a.w, host + at, size_t(c) * 4);
    k_store_words<<<1, 256, 0, st>>>(dst + at, a, c);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace cliff
