// Device-side building blocks shared by the libnqs kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/nqs.h"

#define NQS_WAVE 64

// ---------------------------------------------------------------------------------
// Complex / real scalars. V<T, C> carries an imaginary part only when C is true; with
// C false every operation below reduces to real arithmetic at compile time.
// ---------------------------------------------------------------------------------
template <typename T, bool C>
struct V {
  T re, im;
};

template <typename T, bool C>
__device__ __forceinline__ V<T, C> vmake(T re, T im) {
  V<T, C> r;
  r.re = re;
  r.im = C ? im : T(0);
  return r;
}

// load element idx of an array stored with stride 2 (complex, interleaved) or 1 (real)
template <typename T, bool C, typename S>
__device__ __forceinline__ V<T, C> vload(const S *p, int64_t idx) {
  if constexpr (C)
    return vmake<T, C>(T(p[2 * idx]), T(p[2 * idx + 1]));
  else
    return vmake<T, C>(T(p[idx]), T(0));
}

template <typename T, bool C, typename S>
__device__ __forceinline__ void vstore(S *p, int64_t idx, V<T, C> v) {
  if constexpr (C) {
    p[2 * idx] = S(v.re);
    p[2 * idx + 1] = S(v.im);
  } else {
    p[idx] = S(v.re);
  }
}

template <typename T, bool C>
__device__ __forceinline__ V<T, C> vadd(V<T, C> a, V<T, C> b) {
  return vmake<T, C>(a.re + b.re, C ? a.im + b.im : T(0));
}
template <typename T, bool C>
__device__ __forceinline__ V<T, C> vsub(V<T, C> a, V<T, C> b) {
  return vmake<T, C>(a.re - b.re, C ? a.im - b.im : T(0));
}
template <typename T, bool C>
__device__ __forceinline__ V<T, C> vmul(V<T, C> a, V<T, C> b) {
  if constexpr (C)
    return vmake<T, C>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
  else
    return vmake<T, C>(a.re * b.re, T(0));
}
template <typename T, bool C>
__device__ __forceinline__ V<T, C> vscale(V<T, C> a, T s) {
  return vmake<T, C>(a.re * s, C ? a.im * s : T(0));
}
template <typename T, bool C>
__device__ __forceinline__ V<T, C> vconj(V<T, C> a) {
  return vmake<T, C>(a.re, C ? -a.im : T(0));
}
template <typename T, bool C>
__device__ __forceinline__ T vabs2(V<T, C> a) {
  return C ? a.re * a.re + a.im * a.im : a.re * a.re;
}
template <typename T, bool C, typename U>
__device__ __forceinline__ V<U, C> vcast(V<T, C> a) {
  return vmake<U, C>(U(a.re), U(a.im));
}

// ---------------------------------------------------------------------------------
// Elementary functions of a complex angle z = x + i y, written so that nothing
// overflows for large |x| (e = exp(-2|x|) <= 1):
//   tanh z   = [sgn(x)(1 - e^2) + i 2 e sin 2y] / (1 + e^2 + 2 e cos 2y)
//   ln cosh z = |x| + log(1 + 2 e cos 2y + e^2)/2 - ln 2
//               + i [sgn(x) y + atan2(-sgn(x) e sin 2y, 1 + e cos 2y)]   (mod 2 pi)
// ---------------------------------------------------------------------------------
__device__ __forceinline__ float fexp(float x) { return expf(x); }
__device__ __forceinline__ double fexp(double x) { return exp(x); }
__device__ __forceinline__ float flog1p(float x) { return log1pf(x); }
__device__ __forceinline__ double flog1p(double x) { return log1p(x); }
__device__ __forceinline__ void fsincos(float x, float *s, float *c) { sincosf(x, s, c); }
__device__ __forceinline__ void fsincos(double x, double *s, double *c) { sincos(x, s, c); }
__device__ __forceinline__ float fatan2(float y, float x) { return atan2f(y, x); }
__device__ __forceinline__ double fatan2(double y, double x) { return atan2(y, x); }

// round to the nearest bfloat16 (ties to even), kept in a float; finite inputs only
__device__ __forceinline__ float bf16_round(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xffff0000u);
}

// Exact three-way bf16 split of an FP32 value by truncation: x = h + m + l, h the upper
// 16 bits of x, m those of r = x - h, l = r - m. Both differences are exact in FP32
// (r keeps at most 16 significant bits, l at most 8), so l is itself a bf16 and the
// three parts sum to x exactly. Against a +/-1 operand every product is exact, and a
// bf16 matrix-core contraction with FP32 accumulation gives the FP32 result up to the
// order of the additions.
__device__ __forceinline__ float bf16_rest(float x) {
  return x - __uint_as_float(__float_as_uint(x) & 0xffff0000u);
}
// the upper halves (bf16 truncations) of a and b in one register, a in the low half
__device__ __forceinline__ uint32_t pack_hi(float a, float b) {
  return (__float_as_uint(a) >> 16) | (__float_as_uint(b) & 0xffff0000u);
}
// The bf16 split of an FP32 direction table, the B operand of the JVP on the bf16 matrix
// cores, is stored right after the FP32 table V^T [N][M] (compute precision, es bytes per
// value): 16-bit parts, part p of plane pl of V_ij at
// (((pl * 3 + p) * Np8 / 8 + i / 8) * M + j) * 8 + i % 8, Np8 = N rounded up to 8: the
// eight consecutive sites of one hidden unit are 16 bytes, and consecutive hidden units
// are consecutive 16-byte groups. The entries i >= N are zero.
__host__ __device__ inline int vsplit_np8(int N) { return (N + 7) / 8 * 8; }
__host__ __device__ inline size_t vsplit_offset(int N, int M, size_t es) {
  return (size_t(N) * M * es + 255) / 256 * 256;
}
__host__ __device__ inline size_t vsplit_bytes(int N, int M, int planes) {
  return size_t(planes) * 3 * M * vsplit_np8(N) * 2;
}
template <bool C>
__device__ __forceinline__ void vsplit_store(uint16_t *Vs, int N, int M, int i, int j, float re,
                                             float im) {
  const size_t gp = size_t(vsplit_np8(N) / 8);
#pragma unroll
  for (int pl = 0; pl < (C ? 2 : 1); ++pl) {
    const float x = pl ? im : re;
    const float r = bf16_rest(x), l = bf16_rest(r);
    const size_t o = ((size_t(pl * 3) * gp + i / 8) * M + j) * 8 + i % 8, ps = gp * M * 8;
    Vs[o] = uint16_t(__float_as_uint(x) >> 16);
    Vs[o + ps] = uint16_t(__float_as_uint(r) >> 16);
    Vs[o + 2 * ps] = uint16_t(__float_as_uint(l) >> 16);
  }
}

// reciprocal: the hardware v_rcp_f32 (1 ulp) in single precision, correctly rounded
// division in double
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double frcp(double x) { return 1.0 / x; }

template <typename T, bool C>
__device__ __forceinline__ V<T, C> vtanh(V<T, C> z) {
  T ax = z.re < T(0) ? -z.re : z.re;
  T sg = z.re < T(0) ? T(-1) : T(1);
  T e = fexp(T(-2) * ax);
  if constexpr (C) {
    T s2, c2;
    fsincos(T(2) * z.im, &s2, &c2);
    T d = T(1) + e * e + T(2) * e * c2;
    T inv = frcp(d);
    return vmake<T, C>(sg * (T(1) - e * e) * inv, T(2) * e * s2 * inv);
  } else {
    return vmake<T, C>(sg * (T(1) - e) * frcp(T(1) + e), T(0));
  }
}

template <typename T, bool C>
__device__ __forceinline__ V<T, C> vlncosh(V<T, C> z) {
  const T ln2 = T(0.69314718055994530942);
  T ax = z.re < T(0) ? -z.re : z.re;
  T sg = z.re < T(0) ? T(-1) : T(1);
  T e = fexp(T(-2) * ax);
  if constexpr (C) {
    T s2, c2;
    fsincos(T(2) * z.im, &s2, &c2);
    T re = ax + T(0.5) * flog1p(T(2) * e * c2 + e * e) - ln2;
    T im = sg * z.im + fatan2(-sg * e * s2, T(1) + e * c2);
    return vmake<T, C>(re, im);
  } else {
    return vmake<T, C>(ax + flog1p(e) - ln2 + T(0) * sg, T(0));
  }
}

// ---------------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): 10 rounds, multipliers 0xD2511F53 and
// 0xCD9E8D57, Weyl key increments 0x9E3779B9 and 0xBB67AE85.
// ---------------------------------------------------------------------------------
struct Philox4 {
  uint32_t w[4];
};

__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                 uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
    uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
    uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  Philox4 o;
  o.w[0] = c0;
  o.w[1] = c1;
  o.w[2] = c2;
  o.w[3] = c3;
  return o;
}

// floor(w * n / 2^32)
__device__ __forceinline__ int rng_index(uint32_t w, uint32_t n) {
  return int((uint64_t(w) * uint64_t(n)) >> 32);
}
// (w1 * 2^21 + (w2 >> 11)) * 2^-53 in [0, 1)
__device__ __forceinline__ double rng_uniform(uint32_t w1, uint32_t w2) {
  uint64_t x = (uint64_t(w1) << 21) | uint64_t(w2 >> 11);
  return double(x) * 0x1.0p-53;
}

enum { TAG_PROPOSAL = 0, TAG_INIT = 1, TAG_SWAP = 2, TAG_TARGET = 3 };

// ---------------------------------------------------------------------------------
// Wave-wide reductions (all 64 lanes receive the result).
// ---------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, NQS_WAVE);
  return v;
}

__device__ __forceinline__ int wave_isum(int v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, NQS_WAVE);
  return v;
}

// x = mant * 2^e with mant in [0.5, 1) (mant = 0 for x = 0)
__device__ __forceinline__ float nfrexp(float x, int *e) { return frexpf(x, e); }
__device__ __forceinline__ double nfrexp(double x, int *e) { return frexp(x, e); }
__device__ __forceinline__ float nldexp(float x, int e) { return ldexpf(x, e); }
__device__ __forceinline__ double nldexp(double x, int e) { return ldexp(x, e); }

// product of positive reals kept as mantissa in [0.5, 1) and a base-2 exponent
template <typename T>
__device__ __forceinline__ void wave_prod_norm(T &mant, int &ex) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    T om = __shfl_xor(mant, m, NQS_WAVE);
    int oe = __shfl_xor(ex, m, NQS_WAVE);
    int e2;
    mant = nfrexp(mant * om, &e2);
    ex += oe + e2;
  }
}

// rescale a complex running product by a power of two so that max(|re|, |im|) is in
// [0.5, 1); the exponent moves to ex (exact). Branch-free: a zero product has exponent 0
// and is left as it is.
template <typename T, bool C>
__device__ __forceinline__ void vrenorm(V<T, C> &p, int &ex) {
  T a = p.re < T(0) ? -p.re : p.re;
  if constexpr (C) {
    T b = p.im < T(0) ? -p.im : p.im;
    a = a > b ? a : b;
  }
  int e;
  nfrexp(a, &e);
  e = a > T(0) ? e : 0;
  p.re = nldexp(p.re, -e);
  if constexpr (C) p.im = nldexp(p.im, -e);
  ex += e;
}

// ---------------------------------------------------------------------------------
// DPP butterflies inside each row of 16 lanes (xor 1, xor 2 via quad permutations,
// then rotations by 4 and 8), and the four row totals gathered with readlane.
// ---------------------------------------------------------------------------------
enum { DPP_QP_XOR1 = 0xB1, DPP_QP_XOR2 = 0x4E, DPP_ROR4 = 0x124, DPP_ROR8 = 0x128 };
// lane 15 of each row to the next row, lane 31 to rows 2 and 3 (row_mask selects targets)
enum { DPP_BCAST15 = 0x142, DPP_BCAST31 = 0x143 };

template <int CTRL>
__device__ __forceinline__ int dpp_i(int x) {
  return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f(float x) {
  return __int_as_float(dpp_i<CTRL>(__float_as_int(x)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  int lo = __double2loint(x), hi = __double2hiint(x);
  return __hiloint2double(dpp_i<CTRL>(hi), dpp_i<CTRL>(lo));
}
template <int CTRL>
__device__ __forceinline__ float dpp_v(float x) { return dpp_f<CTRL>(x); }
template <int CTRL>
__device__ __forceinline__ double dpp_v(double x) { return dpp_d<CTRL>(x); }

__device__ __forceinline__ float readlane_v(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
__device__ __forceinline__ double readlane_v(double x, int l) {
  int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
  int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
  return __hiloint2double(hi, lo);
}

// wave-uniform sum (result identical on every lane, fixed order)
template <typename T>
__device__ __forceinline__ T wave_sum_dpp(T x) {
  x += dpp_v<DPP_QP_XOR1>(x);
  x += dpp_v<DPP_QP_XOR2>(x);
  x += dpp_v<DPP_ROR4>(x);
  x += dpp_v<DPP_ROR8>(x);
  return (readlane_v(x, 0) + readlane_v(x, 16)) + (readlane_v(x, 32) + readlane_v(x, 48));
}

// wave-uniform product of positive values given as (mant in [0.5, 1), exponent): returns
// the product mantissa (>= 2^-64, no renormalisation needed) and the summed exponent
template <typename T>
__device__ __forceinline__ T wave_prod_dpp(T mant, int &ex) {
  mant *= dpp_v<DPP_QP_XOR1>(mant);
  ex += dpp_i<DPP_QP_XOR1>(ex);
  mant *= dpp_v<DPP_QP_XOR2>(mant);
  ex += dpp_i<DPP_QP_XOR2>(ex);
  mant *= dpp_v<DPP_ROR4>(mant);
  ex += dpp_i<DPP_ROR4>(ex);
  mant *= dpp_v<DPP_ROR8>(mant);
  ex += dpp_i<DPP_ROR8>(ex);
  ex = (__builtin_amdgcn_readlane(ex, 0) + __builtin_amdgcn_readlane(ex, 16)) +
       (__builtin_amdgcn_readlane(ex, 32) + __builtin_amdgcn_readlane(ex, 48));
  return (readlane_v(mant, 0) * readlane_v(mant, 16)) * (readlane_v(mant, 32) * readlane_v(mant, 48));
}

// wave-uniform complex product of per-lane values p * 2^ex, each normalised by vrenorm;
// the result is renormalised (mantissa with max(|re|, |im|) in [0.5, 1), exponent ex)
template <typename T, bool C, int CTRL>
__device__ __forceinline__ void cprod_step(V<T, C> &p, int &ex) {
  V<T, C> q = vmake<T, C>(dpp_v<CTRL>(p.re), C ? dpp_v<CTRL>(p.im) : T(0));
  ex += dpp_i<CTRL>(ex);
  p = vmul(p, q);
}
template <typename T, bool C>
__device__ __forceinline__ V<T, C> wave_cprod_dpp(V<T, C> p, int &ex) {
  // inside a row: 4 steps, magnitudes stay within [2^-8, 2^4] of the normalised inputs
  cprod_step<T, C, DPP_QP_XOR1>(p, ex);
  cprod_step<T, C, DPP_QP_XOR2>(p, ex);
  cprod_step<T, C, DPP_ROR4>(p, ex);
  cprod_step<T, C, DPP_ROR8>(p, ex);
  vrenorm(p, ex);
  V<T, C> acc = vmake<T, C>(readlane_v(p.re, 0), C ? readlane_v(p.im, 0) : T(0));
  int e = __builtin_amdgcn_readlane(ex, 0);
#pragma unroll
  for (int row = 1; row < 4; ++row) {
    V<T, C> q = vmake<T, C>(readlane_v(p.re, 16 * row), C ? readlane_v(p.im, 16 * row) : T(0));
    e += __builtin_amdgcn_readlane(ex, 16 * row);
    acc = vmul(acc, q);
    vrenorm(acc, e);
  }
  ex = e;
  return acc;
}

template <typename T, bool C>
__device__ __forceinline__ V<T, C> vdiv(V<T, C> a, V<T, C> b) {
  if constexpr (C) {
    T inv = frcp(b.re * b.re + b.im * b.im);
    return vmake<T, C>((a.re * b.re + a.im * b.im) * inv, (a.im * b.re - a.re * b.im) * inv);
  } else {
    return vmake<T, C>(a.re * frcp(b.re), T(0));
  }
}

// wave-local memory ordering for LDS written by one lane and read by others
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------------------------------
// Model data seen by the kernels.
// ---------------------------------------------------------------------------------
struct DevModel {
  int N, M, B0, Btot, ham, move;
  double h;
  const int *bonds;        // [Btot][2], color-0 bonds first
  const double *bond_diag; // [Btot] coefficient of sz_i sz_j on the diagonal
  const double *bond_off;  // [Btot] exchange element (Heisenberg) incl. Marshall sign
};

// Parameter-derived tables, refreshed at the start of each call that needs them.
// Element strides are 2 (complex) or 1 (real) in T; "a"-factors are complex double.
template <typename T>
struct Tables {
  T *Wt;    // [N][M]    W transposed (site-major)
  T *bv;    // [M]       hidden bias
  T *fC;    // [N][M]    cosh(2 W_ji)           (single flip of site i)
  T *fS;    // [N][M]    sinh(2 W_ji)
  T *bC;    // [Btot][M] cosh(2 (W_ji - W_jk))  (exchange on bond (i, k))
  T *bS;    // [Btot][M] sinh(2 (W_ji - W_jk))
  double *fa;  // [2][N]    exp(-2 s a_i),           s = +1 -> row 0, s = -1 -> row 1
  double *ba;  // [2][Btot] exp(-2 s (a_i - a_k)),   s = sigma_i
  double *av;  // [N][2]    a (double, re and im)
  T *Wd;       // [B0][M]   W_ji - W_jk for the color-0 bond (i, k)
};
