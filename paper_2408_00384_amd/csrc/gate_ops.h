// Gate op word of the library's encoded gate streams: the host encoder builds
// it, the gate kernels (single tableau, all-layers-in-LDS, batched) decode it.
//
//   bits  0..23  qubit a
//   bits 24..47  qubit b (two-qubit gates)
//   bits 48..54  single-qubit Clifford applied to a first   (7-bit code, 0 = identity)
//   bits 55..61  single-qubit Clifford applied to b first
//   bits 62..63  two-qubit gate on (a, b) after them: 0 none, 1 CNOT(a -> b), 2 CZ, 3 SWAP
//
// Single-qubit code.  Conjugation by a single-qubit Clifford maps the (x, z)
// bits of a row on its qubit by an invertible 2x2 matrix over GF(2) and flips
// the row's sign by a function of (x, z) that vanishes at (0, 0), which is
// always of the form px x ^ pz z ^ pxz x z:
//   x' = m00 x ^ m01 z,   z' = m10 x ^ m11 z,   r ^= px x ^ pz z ^ pxz (x & z)
// Code bits: 0 = m00 ^ 1, 1 = m01, 2 = m10, 3 = m11 ^ 1, 4 = px, 5 = pz,
// 6 = pxz.  H, S, S^dagger, X, Y, Z and any product of them are such maps
// (the rules of the phase-space method, Sec. 2 via Aaronson & Gottesman), and
// so is their composition, which the host forms before encoding.
//
// Two-qubit rules (after the single-qubit parts):
//   CNOT(a -> b): r ^= x_a z_b ~(x_b ^ z_a);  x_b ^= x_a;  z_a ^= z_b
//   CZ(a, b):     r ^= x_a x_b (z_a ^ z_b);   z_a ^= x_b;  z_b ^= x_a
//   SWAP(a, b):   exchange (x_a, z_a) and (x_b, z_b)
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cliff {

constexpr uint32_t kQubitBits = 24;
constexpr uint64_t kQubitMask = (1ull << kQubitBits) - 1;
constexpr uint32_t kCodeA = 48, kCodeB = 55, kPairShift = 62;
constexpr uint32_t PAIR_NONE = 0, PAIR_CNOT = 1, PAIR_CZ = 2, PAIR_SWAP = 3;

// single-qubit codes of the named gates
constexpr uint32_t SQ_I = 0;
constexpr uint32_t SQ_H = 0b1001111;      // x' = z, z' = x, r ^= x z
constexpr uint32_t SQ_S = 0b1000100;      // z' = x ^ z, r ^= x z
constexpr uint32_t SQ_SDG = 0b1010100;    // z' = x ^ z, r ^= x ^ x z  (= x & ~z)
constexpr uint32_t SQ_X = 0b0100000;      // r ^= z
constexpr uint32_t SQ_Y = 0b0110000;      // r ^= x ^ z
constexpr uint32_t SQ_Z = 0b0010000;      // r ^= x

__host__ __device__ constexpr uint64_t make_op(uint32_t a, uint32_t b, uint32_t ca, uint32_t cb,
                                               uint32_t pair) {
  return uint64_t(a) | (uint64_t(b) << kQubitBits) | (uint64_t(ca) << kCodeA) |
         (uint64_t(cb) << kCodeB) | (uint64_t(pair) << kPairShift);
}
__host__ __device__ inline uint32_t op_a(uint64_t op) { return uint32_t(op & kQubitMask); }
__host__ __device__ inline uint32_t op_b(uint64_t op) { return uint32_t((op >> kQubitBits) & kQubitMask); }
__host__ __device__ inline uint32_t op_ca(uint64_t op) { return uint32_t(op >> kCodeA) & 0x7Fu; }
__host__ __device__ inline uint32_t op_cb(uint64_t op) { return uint32_t(op >> kCodeB) & 0x7Fu; }
__host__ __device__ inline uint32_t op_pair(uint64_t op) { return uint32_t(op >> kPairShift); }
// An op a kernel can apply to an n-qubit tableau: a in range, and for a
// two-qubit gate b in range and distinct from a.
__host__ __device__ inline bool op_valid(uint64_t op, uint32_t n) {
  const uint32_t a = op_a(op), b = op_b(op);
  return a < n && (op_pair(op) == PAIR_NONE || (b < n && b != a));
}

// 128 rows as two 64-bit words (bitwise operators only).
struct alignas(16) U128 {
  uint64_t lo, hi;
};
__device__ __forceinline__ U128 operator&(U128 a, U128 b) { return {a.lo & b.lo, a.hi & b.hi}; }
__device__ __forceinline__ U128 operator^(U128 a, U128 b) { return {a.lo ^ b.lo, a.hi ^ b.hi}; }
__device__ __forceinline__ U128 operator~(U128 a) { return {~a.lo, ~a.hi}; }
__device__ __forceinline__ U128 &operator^=(U128 &a, U128 b) { a = a ^ b; return a; }

// All-ones word if b (0 or 1) is set, else zero (one 32-bit value, repeated).
template <typename T>
__device__ __forceinline__ T mask_if(uint32_t b);
template <>
__device__ __forceinline__ uint32_t mask_if<uint32_t>(uint32_t b) { return 0u - b; }
template <>
__device__ __forceinline__ uint64_t mask_if<uint64_t>(uint32_t b) {
  const uint64_t m = 0u - b;
  return (m << 32) | m;
}
template <>
__device__ __forceinline__ U128 mask_if<U128>(uint32_t b) {
  const uint64_t m = mask_if<uint64_t>(b);
  return {m, m};
}

// Any bitwise function of three words, one v_bitop3 per 32 bits.  LUT is the
// function's value on the inputs (0xF0, 0xCC, 0xAA): bit (4a + 2b + c) of LUT
// is f(a, b, c).
template <uint32_t LUT>
__device__ __forceinline__ uint32_t bop3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, LUT);
}
template <uint32_t LUT>
__device__ __forceinline__ uint64_t bop3(uint64_t a, uint64_t b, uint64_t c) {
  const uint32_t lo = bop3<LUT>(uint32_t(a), uint32_t(b), uint32_t(c));
  const uint32_t hi = bop3<LUT>(uint32_t(a >> 32), uint32_t(b >> 32), uint32_t(c >> 32));
  return (uint64_t(hi) << 32) | lo;
}
template <uint32_t LUT>
__device__ __forceinline__ U128 bop3(U128 a, U128 b, U128 c) {
  return {bop3<LUT>(a.lo, b.lo, c.lo), bop3<LUT>(a.hi, b.hi, c.hi)};
}
constexpr uint32_t LUT_AND3 = 0x80;        // a & b & c
constexpr uint32_t LUT_AND_XOR = 0x6A;     // (a & b) ^ c
constexpr uint32_t LUT_ANDN_XOR = 0x9A;    // (a & ~b) ^ c
constexpr uint32_t LUT_AND_ANDN = 0x40;    // a & b & ~c
constexpr uint32_t LUT_AND_XNOR = 0x90;    // a & ~(b ^ c)

// Apply a single-qubit code to x / z words of rows (32, 64 or 128 rows at once).
template <typename T>
__device__ __forceinline__ void sq_apply(uint32_t c, T &x, T &z, T &racc) {
  auto bit = [c](uint32_t k) { return mask_if<T>((c >> k) & 1u); };   // all-ones if set
  // racc ^= (x & p_x) ^ (z & p_z) ^ (x & z & p_xz)
  racc ^= bop3<LUT_AND_XOR>(z, bit(5), bop3<LUT_AND_XOR>(x, bit(4), bop3<LUT_AND3>(x, z, bit(6))));
  const T nx = bop3<LUT_ANDN_XOR>(x, bit(0), z & bit(1));   // (x & m00) ^ (z & m01)
  const T nz = bop3<LUT_ANDN_XOR>(z, bit(3), x & bit(2));   // (x & m10) ^ (z & m11)
  x = nx;
  z = nz;
}

template <typename T>
__device__ __forceinline__ void pair_apply(uint32_t kind, T &xa, T &za, T &xb, T &zb, T &racc) {
  if (kind == PAIR_CNOT) {
    racc ^= bop3<LUT_AND_ANDN>(xa, zb, xb ^ za);   // xa & zb & ~(xb ^ za)
    xb ^= xa;
    za ^= zb;
  } else if (kind == PAIR_CZ) {
    racc ^= bop3<LUT_AND3>(xa, xb, za ^ zb);       // xa & xb & (za ^ zb)
    za ^= xb;
    zb ^= xa;
  } else if (kind == PAIR_SWAP) {
    const T tx = xa, tz = za;
    xa = xb;
    za = zb;
    xb = tx;
    zb = tz;
  }
}

// ---- host side: composition of single-qubit codes
// (x', z', flip) of code c on input bits (x, z)
inline void sq_eval(uint32_t c, uint32_t x, uint32_t z, uint32_t *xo, uint32_t *zo, uint32_t *f) {
  const uint32_t m00 = ~c & 1u, m01 = (c >> 1) & 1u, m10 = (c >> 2) & 1u, m11 = (~c >> 3) & 1u;
  *xo = (m00 & x) ^ (m01 & z);
  *zo = (m10 & x) ^ (m11 & z);
  *f = (((c >> 4) & 1u) & x) ^ (((c >> 5) & 1u) & z) ^ (((c >> 6) & 1u) & x & z);
}

// Code of "first, then `then`" (both single-qubit codes on one qubit).
inline uint32_t sq_compose(uint32_t first, uint32_t then) {
  uint32_t xo[3], zo[3], f[3];
  const uint32_t in[3][2] = {{1, 0}, {0, 1}, {1, 1}};
  for (int k = 0; k < 3; ++k) {
    uint32_t x1, z1, f1, x2, z2, f2;
    sq_eval(first, in[k][0], in[k][1], &x1, &z1, &f1);
    sq_eval(then, x1, z1, &x2, &z2, &f2);
    xo[k] = x2;
    zo[k] = z2;
    f[k] = f1 ^ f2;
  }
  // linear parts from the images of (1, 0) and (0, 1); flip terms from all three
  const uint32_t m00 = xo[0], m10 = zo[0], m01 = xo[1], m11 = zo[1];
  const uint32_t px = f[0], pz = f[1], pxz = f[2] ^ f[0] ^ f[1];
  return (m00 ^ 1u) | (m01 << 1) | (m10 << 2) | ((m11 ^ 1u) << 3) | (px << 4) | (pz << 5) | (pxz << 6);
}

}  // namespace cliff
