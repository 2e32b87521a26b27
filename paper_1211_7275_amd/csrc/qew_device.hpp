// qew_device.hpp -- device building blocks of the QEW integrator (gfx950).
//
// Counter-based disorder (the paper's memory-free scheme, Sec. IV D): the
// random value at integer point (j, n) of sample `id` is a pure function of
// (seed, j, n, id), so it is regenerated wherever it is needed and never
// stored as an L x M array.
//
// Everything here is __forceinline__ and written with explicit fmaf/fma where
// a fused multiply-add is wanted; the library is built with
// -ffp-contract=off, so the arithmetic of one site update is the same in every
// kernel that calls these functions (fused and one-step kernels produce
// bit-identical states).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qew {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kWeyl0 = 0x9E3779B9u;
constexpr uint32_t kWeyl1 = 0xBB67AE85u;

constexpr int kRF = 0;     // random field, uniform force values, Catmull-Rom
constexpr int kRB = 1;     // random bond, Gaussian potential, Catmull-Rom
constexpr int kRBLin = 2;  // random bond, Gaussian potential, linear spline (Case 3)
constexpr int kRFPc = 3;   // random field, Gaussian forces, no interpolation (Case 4)

// Three-input exclusive or in one VALU instruction (v_bitop3_b32 with the
// truth table of a ^ b ^ c).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32->64
// products with the Weyl-bumped key.  A round is two v_mad_u64_u32 and two
// three-input xors.  The first two rounds keep plain xors: the disorder's
// counters have wave-uniform words (sample id, 0) whose share of those rounds
// the compiler then computes on the scalar unit.
__device__ __forceinline__ void philox4x32_10(uint32_t& x0, uint32_t& x1, uint32_t& x2,
                                              uint32_t& x3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)kPhiloxM0 * (uint64_t)x0;
    const uint64_t p1 = (uint64_t)kPhiloxM1 * (uint64_t)x2;
    const uint32_t h0 = (uint32_t)(p0 >> 32), h1 = (uint32_t)(p1 >> 32);
    const uint32_t y0 = r < 2 ? h1 ^ x1 ^ k0 : xor3(h1, x1, k0);
    const uint32_t y2 = r < 2 ? h0 ^ x3 ^ k1 : xor3(h0, x3, k1);
    x1 = (uint32_t)p1;
    x3 = (uint32_t)p0;
    x0 = y0;
    x2 = y2;
    k0 += kWeyl0;
    k1 += kWeyl1;
  }
}

// The ten round keys in vector registers, for kernels with registers to
// spare: a three-input xor on vector registers issues faster than one with a
// scalar-register operand on gfx950.
struct VectorKeys {
  uint32_t k0[10], k1[10];
};

__device__ __forceinline__ VectorKeys vector_keys(uint32_t k0, uint32_t k1) {
  VectorKeys v;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    v.k0[r] = k0 + (uint32_t)r * kWeyl0;
    v.k1[r] = k1 + (uint32_t)r * kWeyl1;
    asm volatile("" : "+v"(v.k0[r]));
    asm volatile("" : "+v"(v.k1[r]));
  }
  return v;
}

// The same generator with the round keys of `keys`.
__device__ __forceinline__ void philox4x32_10(uint32_t& x0, uint32_t& x1, uint32_t& x2,
                                              uint32_t& x3, const VectorKeys& keys) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)kPhiloxM0 * (uint64_t)x0;
    const uint64_t p1 = (uint64_t)kPhiloxM1 * (uint64_t)x2;
    const uint32_t y0 = xor3((uint32_t)(p1 >> 32), x1, keys.k0[r]);
    const uint32_t y2 = xor3((uint32_t)(p0 >> 32), x3, keys.k1[r]);
    x1 = (uint32_t)p1;
    x3 = (uint32_t)p0;
    x0 = y0;
    x2 = y2;
  }
}

// Raw words of the disorder generator at (j, n): counter (j, (uint32)n, id, 0),
// with n taken modulo the transverse period when there is one.
struct NodeWords {
  uint32_t x0, x1;
};

__device__ __forceinline__ int32_t wrap_cell(int32_t n, int32_t period) {
  if (period <= 0) return n;
  int32_t m = n % period;
  return m < 0 ? m + period : m;
}

__device__ __forceinline__ NodeWords node_words(uint32_t j, int32_t n, uint32_t id, uint32_t k0,
                                                uint32_t k1) {
  uint32_t x0 = j, x1 = (uint32_t)n, x2 = id, x3 = 0u;
  philox4x32_10(x0, x1, x2, x3, k0, k1);
  return {x0, x1};
}

__device__ __forceinline__ NodeWords node_words(uint32_t j, int32_t n, uint32_t id, const VectorKeys& keys) {
  uint32_t x0 = j, x1 = (uint32_t)n, x2 = id, x3 = 0u;
  philox4x32_10(x0, x1, x2, x3, keys);
  return {x0, x1};
}

// Random-field force value: 24 random bits m = x0 >> 8 mapped to the odd
// grid (2m + 1 - 2^24) / 2^24, uniform in (-1, 1).  (x0 >> 7) | 1 == 2m + 1.
// Exact in FP32 and FP64.
__device__ __forceinline__ int32_t rf_odd(uint32_t x0) {
  return (int32_t)((x0 >> 7) | 1u) - (1 << 24);
}

// Random-bond potential value: Box-Muller (cosine branch) on
// U1 = (2a + 1) / 2^24, U2 = (2b + 1) / 2^24, a = x0 >> 9, b = x1 >> 9;
// (x >> 8) | 1 == 2a + 1.  Both uniforms are exact in FP32 and FP64.
__device__ __forceinline__ float rb_value_f32(uint32_t x0, uint32_t x1) {
  const float u1 = (float)((x0 >> 8) | 1u) * 0x1p-24f;
  const float u2 = (float)((x1 >> 8) | 1u) * 0x1p-24f;
  // -2 ln u1 = -2 ln(2) log2(u1); v_log_f32 is log2, v_cos_f32 takes revolutions.
  const float radius = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u1));
  return radius * __builtin_amdgcn_cosf(u2);
}

__device__ __forceinline__ double rb_value_f64(uint32_t x0, uint32_t x1) {
  const double u1 = (double)((x0 >> 8) | 1u) * 0x1p-24;
  const double u2 = (double)((x1 >> 8) | 1u) * 0x1p-24;
  const double radius = sqrt(-2.0 * log(u1));
  const double angle = 2.0 * 3.14159265358979323846 * u2;
  return radius * cos(angle);
}

// Node value at (j, n): uniform for kRF, N(0, 1) (Box-Muller) for the other
// kinds; n is wrapped by the transverse period `period` (0: none).
template <int KIND>
__device__ __forceinline__ float node_f32(uint32_t j, int32_t n, uint32_t id, uint32_t k0,
                                          uint32_t k1, int32_t period) {
  const NodeWords w = node_words(j, wrap_cell(n, period), id, k0, k1);
  if constexpr (KIND == kRF) {
    return (float)rf_odd(w.x0) * 0x1p-24f;
  } else {
    return rb_value_f32(w.x0, w.x1);
  }
}

// The same with the round keys of `keys` (vector registers).
template <int KIND>
__device__ __forceinline__ float node_f32(uint32_t j, int32_t n, uint32_t id, const VectorKeys& keys,
                                          int32_t period) {
  const NodeWords w = node_words(j, wrap_cell(n, period), id, keys);
  if constexpr (KIND == kRF) {
    return (float)rf_odd(w.x0) * 0x1p-24f;
  } else {
    return rb_value_f32(w.x0, w.x1);
  }
}

template <int KIND>
__device__ __forceinline__ double node_f64(uint32_t j, int32_t n, uint32_t id, uint32_t k0,
                                           uint32_t k1, int32_t period) {
  const NodeWords w = node_words(j, wrap_cell(n, period), id, k0, k1);
  if constexpr (KIND == kRF) {
    return (double)rf_odd(w.x0) * 0x1p-24;
  } else {
    return rb_value_f64(w.x0, w.x1);
  }
}

template <int KIND>
__device__ __forceinline__ double node_f64(uint32_t j, int32_t n, uint32_t id, const VectorKeys& keys,
                                           int32_t period) {
  const NodeWords w = node_words(j, wrap_cell(n, period), id, keys);
  if constexpr (KIND == kRF) {
    return (double)rf_odd(w.x0) * 0x1p-24;
  } else {
    return rb_value_f64(w.x0, w.x1);
  }
}

// ---------------------------------------------------------------------------
// Catmull-Rom spline through p0..p3 at nodes -1, 0, 1, 2, at s in [0, 1].
// value(s) = p1 + s (a1 + s (a2 + s a3)),  slope(s) = a1 + s (2 a2 + 3 a3 s),
//   a1 = (p2 - p0) / 2, a2 = p0 - 5/2 p1 + 2 p2 - 1/2 p3,
//   a3 = 3/2 (p1 - p2) + 1/2 (p3 - p0).
// RF uses the value, RB the slope (F_p = -dU/du).
//
// spline_coef returns the polynomial in s of  f + g * (value or slope),  with
// g = +strength (RF) or -strength (RB) and f the drive, so one Horner
// evaluation (spline_eval) gives the drive plus the pinning force:
//   RF: {x, y, z, w} = {f + g p1, g a1, g a2, g a3}         (cubic)
//   RB: {x, y, z, w} = {f + g a1, g 2 a2, g 3 a3, unused}   (quadratic)
// The coefficients of a cell are computed once and evaluated every step;
// every kernel goes through these two functions, so a cached coefficient set
// gives exactly the force a fresh evaluation gives.
// ---------------------------------------------------------------------------
//   Case 3 (kRBLin): {f + g (p2 - p1), 0, 0, 0} with g = -strength, constant in the cell;
//   Case 4 (kRFPc):  {f + g p1, 0, 0, 0} with g = +strength.
template <int KIND>
__device__ __forceinline__ float4 spline_coef(float p0, float p1, float p2, float p3, float g,
                                              float f) {
  if constexpr (KIND == kRBLin) {
    return make_float4(fmaf(g, p2 - p1, f), 0.0f, 0.0f, 0.0f);
  } else if constexpr (KIND == kRFPc) {
    return make_float4(fmaf(g, p1, f), 0.0f, 0.0f, 0.0f);
  }
  const float a1 = 0.5f * (p2 - p0);
  const float d30 = p3 - p0;
  const float d12 = p1 - p2;
  if constexpr (KIND == kRF) {
    const float a2 = fmaf(-0.5f, p3, fmaf(2.0f, p2, fmaf(-2.5f, p1, p0)));
    const float a3 = fmaf(1.5f, d12, 0.5f * d30);
    return make_float4(fmaf(g, p1, f), g * a1, g * a2, g * a3);
  } else {
    const float b2 = fmaf(-1.0f, p3, fmaf(4.0f, p2, fmaf(-5.0f, p1, 2.0f * p0)));
    const float b3 = fmaf(4.5f, d12, 1.5f * d30);
    return make_float4(fmaf(g, a1, f), g * b2, g * b3, 0.0f);
  }
}

template <int KIND>
__device__ __forceinline__ float spline_eval(const float4& a, float s) {
  if constexpr (KIND == kRF) {
    return fmaf(s, fmaf(s, fmaf(s, a.w, a.z), a.y), a.x);
  } else if constexpr (KIND == kRB) {
    return fmaf(s, fmaf(s, a.z, a.y), a.x);
  } else {
    return a.x;  // piecewise constant in the cell
  }
}

// Sign of the node-value scale: +strength for force values, -strength for
// potential values (F_p = -dU/du).
template <int KIND>
__device__ __forceinline__ float kind_sign() {
  return (KIND == kRF || KIND == kRFPc) ? 1.0f : -1.0f;
}

// FP64 form, same operation order as the textbook polynomial
// 1/2 [2 p1 + (p2 - p0) s + (2p0 - 5p1 + 4p2 - p3) s^2 + (-p0 + 3p1 - 3p2 + p3) s^3];
// Case 3: -(p2 - p1); Case 4: p1 (p scaled by strength).
template <int KIND>
__device__ __forceinline__ double spline_f64(const double p[4], double s) {
  if constexpr (KIND == kRBLin) {
    return -(p[2] - p[1]);
  } else if constexpr (KIND == kRFPc) {
    return p[1];
  }
  const double c1 = p[2] - p[0];
  const double c2 = 2.0 * p[0] - 5.0 * p[1] + 4.0 * p[2] - p[3];
  const double c3 = -p[0] + 3.0 * p[1] - 3.0 * p[2] + p[3];
  if constexpr (KIND == kRF) {
    const double c0 = 2.0 * p[1];
    return 0.5 * (c0 + s * (c1 + s * (c2 + s * c3)));
  } else {
    return -(0.5 * (c1 + s * (2.0 * c2 + s * (3.0 * c3))));
  }
}

// ---------------------------------------------------------------------------
// Site updates.
// ---------------------------------------------------------------------------
struct SplitPhys {
  float c;        // elastic constant
  float dt;       // time step
  float sgn_str;  // +strength (RF) or -strength (RB)
};

// Total force of Eq. (1) on a split site (cell c, offset r) with neighbours
// (cl, rl), (cr, rr); `a` holds the coefficients of f + F_p of its cell.  The
// integer part of the Laplacian is exact; the offsets carry the fraction
// ((rl + rr) - 2 r rounded once: 2 r is exact).
template <int KIND>
__device__ __forceinline__ float split_force(int32_t c, float r, int32_t cl, float rl, int32_t cr,
                                             float rr, const float4& a, float cel) {
  const float lap = (float)((cr - c) - (c - cl)) + fmaf(-2.0f, r, rl + rr);
  return fmaf(cel, lap, spline_eval<KIND>(a, r));
}

// Euler update of a split site: r' = r + dt F, then whole units move into the
// cell.  The offset stays in [0, 1]: it reaches exactly 1 only when r + dt F
// is a negative number above -2^-25 (r' = 1 - |r + dt F| rounds to 1); the
// site then sits at the right end of its cell, where the spline equals the
// next cell's left end.
__device__ __forceinline__ float split_advance(float& r, float F, float dt) {
  const float rn = fmaf(dt, F, r);
  const float fl = floorf(rn);
  r = rn - fl;
  return fl;  // cells moved
}

struct PlainPhys {
  double c, dt, strength;
};

// Total force of Eq. (1) in FP64: ((c * lap) + f) + F_p with all four nodes
// regenerated (the plain path).
template <int KIND, class Keys>
__device__ __forceinline__ double plain_force(double ul, double u, double ur, uint32_t j,
                                              uint32_t id, const Keys& keys, double f,
                                              int32_t period, const PlainPhys& ph) {
  const double lap = (ur + ul) - 2.0 * u;
  double fp = 0.0;
  if (ph.strength != 0.0) {
    const double nf = floor(u);
    const int32_t n = (int32_t)nf;
    const double s = u - nf;
    double p[4] = {0.0, 0.0, 0.0, 0.0};
    // Catmull-Rom needs nodes n-1..n+2, Case 3 n..n+1, Case 4 n.
    constexpr int lo = (KIND == kRF || KIND == kRB) ? 0 : 1;
    constexpr int hi = (KIND == kRF || KIND == kRB) ? 4 : (KIND == kRBLin ? 3 : 2);
#pragma unroll
    for (int i = lo; i < hi; ++i) p[i] = ph.strength * node_f64<KIND>(j, n - 1 + i, id, keys, period);
    fp = spline_f64<KIND>(p, s);
  }
  return ((ph.c * lap) + f) + fp;
}

// ---------------------------------------------------------------------------
// Wave-level helpers (wave64).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

}  // namespace qew
