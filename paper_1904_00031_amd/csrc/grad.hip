// Jacobian products of the RBM log-derivatives on the matrix cores.
//
// O_sk = d log psi(s_s) / d p_k: O_a_i = s_i, O_b_j = t_j, O_W_ji = t_j s_i with
// t_j = tanh(theta_j) (Sec. 2.2.5, analytic RBM derivatives). Both products are built
// from dense contractions over the spin matrix S [n x N] (entries +/-1, exact in every
// precision) and theta is recomputed from S by the same contraction, so the [n x P]
// matrix O is never formed:
//   JVP  y_s = sum_i s_si va_i + sum_j t_sj (vb_j + (S V^T)_sj)      (theta = S W^T + b)
//   VJP  g_W = Z^T S, g_b = colsum(Z), g_a = S^T u,  Z_sj = conj(t_sj) u_s.
// Each wavefront owns 16 samples; the matrix-core instruction is the 16x16x4 FP32 or
// FP64 MFMA (A: lane l holds A[l%16][l/16]; B: B[l/16][l%16]). Accumulator rows differ:
// FP32 lane l register r holds D[4(l/16)+r][l%16], FP64 holds D[l/16+4r][l%16].
#include <type_traits>

#include "internal.hpp"

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

namespace {

template <typename T>
struct MF;
template <>
struct MF<float> {
  typedef floatx4 acc;
  static __device__ __forceinline__ acc mma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // accumulator row held by lane group hi (= lane / 16), register r
  static __device__ __forceinline__ int row(int hi, int r) { return 4 * hi + r; }
};
template <>
struct MF<double> {
  typedef doublex4 acc;
  static __device__ __forceinline__ acc mma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int hi, int r) { return hi + 4 * r; }
};

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t rup(int64_t a, int64_t b) { return cdiv(a, b) * b; }

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
// 16x16x32 bf16 MFMA, FP32 accumulate. A: lane l holds A[l%16][8(l/16) .. 8(l/16)+7];
// B: lane l holds B[8(l/16) .. 8(l/16)+7][l%16]; D as the 16x16x4 FP32 instruction.
// Element e of a register quad is bits 16e .. 16e+15 (dword e/2, low half first).
__device__ __forceinline__ floatx4 mfma_bf16(uint4 a, uint4 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                 __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// T rows of FP32 models: element idx of [n][M] as FP32 values, or (TB, the BF16 form,
// whose rows are bfloat16 by definition) as bfloat16 (re, im) pairs of 4 bytes (2 real)
template <typename T, bool C, bool TB>
__device__ __forceinline__ V<T, C> tload(const T *__restrict__ Tm, int64_t idx) {
  static_assert(!TB || sizeof(T) == 4, "bfloat16 T rows belong to FP32 models");
  if constexpr (!TB) {
    return vload<T, C>(Tm, idx);
  } else if constexpr (C) {
    const uint32_t w = reinterpret_cast<const uint32_t *>(Tm)[idx];
    return vmake<float, true>(__uint_as_float(w << 16), __uint_as_float(w & 0xffff0000u));
  } else {
    const uint32_t h = reinterpret_cast<const unsigned short *>(Tm)[idx];
    return vmake<float, false>(__uint_as_float(h << 16), 0.f);
  }
}

// ---------------------------------------------------------------------------------
// Direction v (double, packed like the parameters) -> compute-precision tables.
// ---------------------------------------------------------------------------------
template <typename T, bool C>
__global__ void k_prep_dir(int N, int M, const double *__restrict__ v, T *Vt, T *vb,
                           double *va, int split) {
  // FP32 with split: the bf16 split of V^T follows V^T (its padding sites i in [N, Np8)
  // zeroed here)
  const bool SPLIT = sizeof(T) == 4 && split;
  uint16_t *Vs = reinterpret_cast<uint16_t *>(reinterpret_cast<char *>(Vt) +
                                              vsplit_offset(N, M, sizeof(T) * (C ? 2 : 1)));
  const int np = vsplit_np8(N);
  const int64_t pad = SPLIT ? int64_t(C ? 2 : 1) * 3 * M * (np - N) : 0;
  const int64_t total = int64_t(N) * M + M + N + pad;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    if (e < int64_t(N) * M) {
      int j = int(e / N), i = int(e % N);  // read v_W row-major (j, i)
      const V<T, C> x = vcast<double, C, T>(vload<double, C>(v, N + M + e));
      vstore<T, C>(Vt, int64_t(i) * M + j, x);
      if (SPLIT) vsplit_store<C>(Vs, N, M, i, j, float(x.re), C ? float(x.im) : 0.f);
    } else if (e >= int64_t(N) * M + M + N) {
      const int64_t q = e - (int64_t(N) * M + M + N);  // padding entry (plane-part, j, site)
      const int i = N + int(q % (np - N));
      const int64_t r = q / (np - N);
      const int64_t pp = r / M, j = r % M;
      Vs[((pp * (np / 8) + i / 8) * M + j) * 8 + i % 8] = 0;
    } else if (e < int64_t(N) * M + M) {
      int j = int(e - int64_t(N) * M);
      vstore<T, C>(vb, j, vcast<double, C, T>(vload<double, C>(v, N + j)));
    } else {
      int i = int(e - int64_t(N) * M - M);
      V<double, C> x = vload<double, C>(v, i);
      va[2 * i] = x.re;
      va[2 * i + 1] = C ? x.im : 0.0;
    }
  }
}

// ---------------------------------------------------------------------------------
// T[s][j] = tanh(b_j + sum_i W_ji s_si): theta tile by MFMA (A = spins, B = W^T), tanh in
// the epilogue. Grid (ceil(n/64), hidden chunks of JT tiles); 16 samples per wavefront.
// ---------------------------------------------------------------------------------
// hidden tiles per block of the theta/tanh and JVP kernels (accumulators per wavefront):
// 8 for real FP32, 4 otherwise
template <typename T, bool C>
struct Chunk {
  static constexpr int JT = (sizeof(T) == 8 || C) ? 4 : 8;
};

// spins s0 s1 (bytes 0 and 2 of u, +/-1 or 0) -> two bf16 in one dword
__device__ __forceinline__ uint32_t spin_pair_bf16(uint32_t u) {
  return ((u << 8) & 0x80008000u) | ((u & 0x00010001u) * 0x3f80u);
}
__device__ __forceinline__ uint4 spins8_bf16(uint32_t a, uint32_t b) {
  return make_uint4(spin_pair_bf16((a & 0xffu) | ((a & 0xff00u) << 8)),
                    spin_pair_bf16(((a >> 16) & 0xffu) | ((a >> 8) & 0xff0000u)),
                    spin_pair_bf16((b & 0xffu) | ((b & 0xff00u) << 8)),
                    spin_pair_bf16(((b >> 16) & 0xffu) | ((b >> 8) & 0xff0000u)));
}

template <typename T, bool C>
__device__ __forceinline__ void k_theta_tanh_body(int BX, int BY, int BZ, int GX, int N, int M,
                                                  int64_t n, const int8_t *__restrict__ sigma,
                                                  const T *__restrict__ Wt,
                                                  const T *__restrict__ bv, int quant, int wbf,
                                                  T *Tout) {
  typedef typename MF<T>::acc Acc;
  constexpr int JT = Chunk<T, C>::JT;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int lo = lane & 15, hi = lane >> 4;
  const int64_t s0 = int64_t(BX) * 64 + wid * 16;
  const int jt0 = BY * JT;
  const int64_t rowA = s0 + lo;
  const bool rowA_ok = rowA < n;
  const int8_t *srow = sigma + (rowA_ok ? rowA : 0) * N;
  Acc tr[JT], ti[JT];
#pragma unroll
  for (int a = 0; a < JT; ++a) {
    tr[a] = Acc{0, 0, 0, 0};
    ti[a] = Acc{0, 0, 0, 0};
  }
  // FP32 / BF16 forms on the bf16 matrix cores (16x16x32) for the BF16 form and for FP32
  // models with at least 128 sites (fewer sites pad the 32-site steps and the three parts
  // of FP32 weights cost more than the FP32 instruction saves); the others below
  bool bf16_cores = false;
  if constexpr (sizeof(T) == 4) bf16_cores = wbf || N >= 128;
  if constexpr (sizeof(T) == 4) {
    if (bf16_cores) {
      // the spins are exact in bf16 and so is each weight of the BF16 form (wbf); an FP32
      // weight is split exactly into three bf16 parts (h, m, l), so every product is exact
      // and the sums are FP32, as on the FP32 matrix cores. Per step of 32 sites: lane
      // (lo, hi) holds the spins of sample s0 + lo at sites k0 + 8 hi .. + 7 (A) and the
      // weights of those sites at unit (jt0 + q) 16 + lo (B).
      const bool al8 = (N & 7) == 0 && (reinterpret_cast<uintptr_t>(sigma) & 7) == 0;
      const int nparts = wbf ? 1 : 3;
      for (int k0 = 0; k0 < N; k0 += 32) {
        const int kb = k0 + 8 * hi;
        uint32_t sa = 0, sb = 0;  // spin bytes (+1 / -1, 0 past N and past n)
        if (rowA_ok && kb < N) {
          if (al8) {
            const uint2 w = *reinterpret_cast<const uint2 *>(srow + kb);
            sa = w.x;
            sb = w.y;
          } else {
  #pragma unroll
            for (int e = 0; e < 8; ++e) {
              const uint32_t x = kb + e < N ? uint32_t(uint8_t(srow[kb + e])) : 0u;
              if (e < 4) sa |= x << (8 * e);
              else sb |= x << (8 * (e - 4));
            }
          }
        }
        const uint4 av = spins8_bf16(sa, sb);
  #pragma unroll
        for (int q = 0; q < JT; ++q) {
          const int j = (jt0 + q) * 16 + lo;
          float wr[8], wi[8];
  #pragma unroll
          for (int e = 0; e < 8; ++e) {
            const int k = kb + e;
            const bool ok = k < N && j < M;
            const V<float, C> x = vload<float, C>(Wt, ok ? int64_t(k) * M + j : 0);
            wr[e] = ok ? x.re : 0.f;
            wi[e] = ok ? (C ? x.im : 0.f) : 0.f;
          }
          for (int part = 0; part < nparts; ++part) {
            const uint4 br = make_uint4(pack_hi(wr[0], wr[1]), pack_hi(wr[2], wr[3]),
                                        pack_hi(wr[4], wr[5]), pack_hi(wr[6], wr[7]));
            tr[q] = mfma_bf16(av, br, tr[q]);
            if constexpr (C) {
              const uint4 bi = make_uint4(pack_hi(wi[0], wi[1]), pack_hi(wi[2], wi[3]),
                                          pack_hi(wi[4], wi[5]), pack_hi(wi[6], wi[7]));
              ti[q] = mfma_bf16(av, bi, ti[q]);
            }
            if (part + 1 < nparts) {
#pragma unroll
              for (int e = 0; e < 8; ++e) {
                wr[e] = bf16_rest(wr[e]);
                if constexpr (C) wi[e] = bf16_rest(wi[e]);
              }
            }
          }
        }
      }
    }
  }
  if (!bf16_cores) {
    // k outer, tiles inner: the A operand and the JT weight loads of a step are issued
    // together (clamped addresses, selects instead of branches)
#pragma unroll 2
    for (int k0 = 0; k0 < N; k0 += 4) {
      const int k = k0 + hi;
      const bool kok = k < N;
      const int8_t sv = srow[kok ? k : 0];
      const T a = (rowA_ok && kok) ? T(sv) : T(0);
      V<T, C> w[JT];
#pragma unroll
      for (int q = 0; q < JT; ++q) {
        const int j = (jt0 + q) * 16 + lo;
        const bool ok = kok && j < M;
        const V<T, C> x = vload<T, C>(Wt, ok ? int64_t(k) * M + j : 0);
        w[q] = ok ? x : vmake<T, C>(T(0), T(0));
      }
#pragma unroll
      for (int q = 0; q < JT; ++q) {
        tr[q] = MF<T>::mma(a, w[q].re, tr[q]);
        if constexpr (C) ti[q] = MF<T>::mma(a, w[q].im, ti[q]);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < JT; ++q) {
    const int j = (jt0 + q) * 16 + lo;
    if (j >= M) continue;
    const V<T, C> bb = vload<T, C>(bv, j);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = s0 + MF<T>::row(hi, r);
      if (row < n) {
        V<T, C> th = vmake<T, C>(tr[q][r] + bb.re, C ? ti[q][r] + bb.im : T(0));
        V<T, C> tv = vtanh<T, C>(th);
        if (quant) {  // BF16 form: the Jacobian contractions see bfloat16 tanh(theta)
          tv.re = T(bf16_round(float(tv.re)));
          if (C) tv.im = T(bf16_round(float(tv.im)));
        }
        if (sizeof(T) == 4 && quant == 2) {  // stored as bfloat16 (exact: rounded above)
          const uint32_t hr = __float_as_uint(float(tv.re)) >> 16;
          if constexpr (C)
            reinterpret_cast<uint32_t *>(Tout)[row * M + j] =
                hr | (__float_as_uint(float(tv.im)) & 0xffff0000u);
          else
            reinterpret_cast<unsigned short *>(Tout)[row * M + j] = (unsigned short)hr;
        } else {
          vstore<T, C>(Tout, row * M + j, tv);
        }
      }
    }
  }
}

template <typename T, bool C>
__global__ __launch_bounds__(256) void k_theta_tanh(int N, int M, int64_t n,
                                                     const int8_t *__restrict__ sigma,
                                                     const T *__restrict__ Wt,
                                                     const T *__restrict__ bv, int quant,
                                                     int wbf, T *Tout) {
  k_theta_tanh_body<T, C>(blockIdx.x, blockIdx.y, 0, 0, N, M, n, sigma, Wt, bv, quant, wbf,
                          Tout);
}

// ---------------------------------------------------------------------------------
// JVP with stored T: y_s = sum_i s_si va_i + sum_j T_sj (vb_j + (S V^T)_sj).
// Grid (ceil(n/64), hidden chunks). Writes ypart[chunk][s] (complex double).
// ---------------------------------------------------------------------------------
template <typename T, bool C>
__device__ __forceinline__ void k_jvp_body(int BX, int BY, int BZ, int GX, int N, int M,
                                           int64_t n, const int8_t *__restrict__ sigma,
                                           const T *__restrict__ Tm, const T *__restrict__ Vt,
                                           const T *__restrict__ vb,
                                           const double *__restrict__ va, double *ypart,
                                           const int *skip) {
  if (skip && *skip) return;
  typedef typename MF<T>::acc Acc;
  constexpr int JT = Chunk<T, C>::JT;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int lo = lane & 15, hi = lane >> 4;
  const int64_t s0 = int64_t(BX) * 64 + wid * 16;
  const int jc = BY;
  const int jt0 = jc * JT;
  const int64_t rowA = s0 + lo;
  const bool rowA_ok = rowA < n;
  const int8_t *srow = sigma + (rowA_ok ? rowA : 0) * N;
  // the T entries of every tile are loaded first; they arrive during the contraction
  V<T, C> tv[JT][4];
#pragma unroll
  for (int q = 0; q < JT; ++q) {
    const int j = (jt0 + q) * 16 + lo;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = s0 + MF<T>::row(hi, r);
      const bool ok = j < M && row < n;
      const V<T, C> x = vload<T, C>(Tm, ok ? row * M + j : 0);
      tv[q][r] = ok ? x : vmake<T, C>(T(0), T(0));
    }
  }
  Acc xr[JT], xi[JT];
#pragma unroll
  for (int q = 0; q < JT; ++q) {
    xr[q] = Acc{0, 0, 0, 0};
    xi[q] = Acc{0, 0, 0, 0};
  }
#pragma unroll 2
  for (int k0 = 0; k0 < N; k0 += 4) {
    const int k = k0 + hi;
    const bool kok = k < N;
    const int8_t sv = srow[kok ? k : 0];
    const T a = (rowA_ok && kok) ? T(sv) : T(0);
    V<T, C> v[JT];
#pragma unroll
    for (int q = 0; q < JT; ++q) {
      const int j = (jt0 + q) * 16 + lo;
      const bool ok = kok && j < M;
      const V<T, C> x = vload<T, C>(Vt, ok ? int64_t(k) * M + j : 0);
      v[q] = ok ? x : vmake<T, C>(T(0), T(0));
    }
#pragma unroll
    for (int q = 0; q < JT; ++q) {
      xr[q] = MF<T>::mma(a, v[q].re, xr[q]);
      if constexpr (C) xi[q] = MF<T>::mma(a, v[q].im, xi[q]);
    }
  }
  V<T, C> yp[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) yp[r] = vmake<T, C>(T(0), T(0));
#pragma unroll
  for (int q = 0; q < JT; ++q) {
    const int j = (jt0 + q) * 16 + lo;
    const V<T, C> vbj = j < M ? vload<T, C>(vb, j) : vmake<T, C>(T(0), T(0));
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      V<T, C> x = vmake<T, C>(xr[q][r] + vbj.re, C ? xi[q][r] + vbj.im : T(0));
      yp[r] = vadd(yp[r], vmul(tv[q][r], x));
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
#pragma unroll
    for (int m = 1; m < 16; m <<= 1) {
      yp[r].re += __shfl_xor(yp[r].re, m, 64);
      if constexpr (C) yp[r].im += __shfl_xor(yp[r].im, m, 64);
    }
  }
  // visible term of chunk 0: sample s0 + lo split over its four lane groups by site
  double vr = 0.0, vi = 0.0;
  if (jc == 0 && rowA_ok) {
    for (int i = hi; i < N; i += 4) {
      const double x = double(srow[i]);
      vr += va[2 * i] * x;
      vi += va[2 * i + 1] * x;
    }
  }
  vr += __shfl_xor(vr, 16, 64);
  vi += __shfl_xor(vi, 16, 64);
  vr += __shfl_xor(vr, 32, 64);
  vi += __shfl_xor(vi, 32, 64);
  double var[4], vai[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    var[r] = __shfl(vr, MF<T>::row(hi, r), 64);
    vai[r] = __shfl(vi, MF<T>::row(hi, r), 64);
  }
  if (lo == 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = s0 + MF<T>::row(hi, r);
      if (row >= n) continue;
      ypart[2 * (int64_t(jc) * n + row)] = double(yp[r].re) + var[r];
      ypart[2 * (int64_t(jc) * n + row) + 1] = (C ? double(yp[r].im) : 0.0) + vai[r];
    }
  }
}

// ---------------------------------------------------------------------------------
// FP32 JVP on the bf16 matrix cores: X = S V^T against the exact three-part bf16 split
// of V stored after V^T (k group g of 8 = part g % 3 of sites 8 (g / 3) .. + 7), then
// y_s = sum_j t_sj (vb_j + X_sj) + sum_i s_si va_i. A block of four wavefronts covers
// CW hidden chunks (JT tiles of 16) and 64 (4 / CW) samples: wavefront w takes chunk
// BY CW + w % CW and the 64 samples of set w / CW as four 16-sample groups, so each
// 16-byte load of the split feeds four MFMAs. The block's spins are staged in LDS as
// bf16 (+1 = 0x3f80, -1 = 0xbf80, zero past N and past n), one window of 256 / sets
// sites at a time. Writes ypart[chunk][s] (complex double); chunk 0 adds the visible
// term, summed in FP64 by one lane per sample.
// ---------------------------------------------------------------------------------
constexpr int kJvpLdsWords = 9216;  // 256 rows x 144 B, 128 x 272 B or 64 x 528 B

inline int jvp32_cw(int jchunks) { return jchunks >= 3 ? 4 : (jchunks == 2 ? 2 : 1); }

template <bool C, bool TB = false>
__device__ __forceinline__ void k_jvp32_body(int BX, int BY, int CW, int jchunks, int N, int M,
                                             int64_t n, const int8_t *__restrict__ sigma,
                                             const float *__restrict__ Tm,
                                             const float *__restrict__ Vt,
                                             const float *__restrict__ vb,
                                             const double *__restrict__ va, double *ypart,
                                             const int *skip) {
  if (skip && *skip) return;
  constexpr int JT = Chunk<float, C>::JT, PL = C ? 2 : 1;
  __shared__ __align__(16) uint32_t sl[kJvpLdsWords];
  __shared__ double2 ysh[4][64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int lo = lane & 15, hi = lane >> 4;
  const int SB = 4 / CW, rows = 64 * SB;
  const int wn = 256 / SB, WG = wn / 8;
  // staged row: WG slots of 8 sites (16 bytes) and one zero slot read by idle k groups
  const int kRowW = 4 * (WG + 1);
  const int chunk = BY * CW + wid % CW, set = wid / CW;
  const bool active = chunk < jchunks;
  const int64_t sb0 = int64_t(BX) * rows, s0 = sb0 + 64 * set;
  const uint4 *Vs = reinterpret_cast<const uint4 *>(
      reinterpret_cast<const char *>(Vt) + vsplit_offset(N, M, sizeof(float) * (C ? 2 : 1)));
  const int GP = vsplit_np8(N) / 8;
  const uint32_t plane = uint32_t(3 * GP) * uint32_t(M);  // uint4 units per plane
  uint32_t jcl[JT];
#pragma unroll
  for (int q = 0; q < JT; ++q) {
    const int j = (chunk * JT + q) * 16 + lo;
    jcl[q] = uint32_t(j < M ? j : M - 1);
  }
  floatx4 acc[4][JT][PL];
#pragma unroll
  for (int g = 0; g < 4; ++g)
#pragma unroll
    for (int q = 0; q < JT; ++q)
#pragma unroll
      for (int pl = 0; pl < PL; ++pl) acc[g][q][pl] = floatx4{0.f, 0.f, 0.f, 0.f};
  const bool vis = active && chunk == 0;
  double vr = 0.0, vi = 0.0;  // visible term of sample s0 + lane
  const bool al8 = (N & 7) == 0 && (reinterpret_cast<uintptr_t>(sigma) & 7) == 0;
  const bool al4 = (N & 3) == 0 && (reinterpret_cast<uintptr_t>(sigma) & 3) == 0;
  for (int wg0 = 0; wg0 < GP; wg0 += WG) {
    const int GPw = GP - wg0 < WG ? GP - wg0 : WG;
    const int c0 = 8 * wg0;
    if (wg0 > 0) __syncthreads();
    // stage rows [sb0, sb0 + rows) x sites [c0, c0 + 8 GPw), 8 sites per item; the last
    // item of a row clears its zero slot
    for (int e = threadIdx.x; e < rows * (GPw + 1); e += 256) {
      const int r = e / (GPw + 1), c = e - r * (GPw + 1);
      const int64_t row = sb0 + r;
      const int col = c0 + 8 * c;
      uint32_t a = 0, b = 0;
      if (row < n && c < GPw) {
        const int8_t *src = sigma + row * N + col;
        if (al8) {
          const uint2 w = *reinterpret_cast<const uint2 *>(src);
          a = w.x;
          b = w.y;
        } else if (al4) {
          a = *reinterpret_cast<const uint32_t *>(src);
          if (col + 4 < N) b = *reinterpret_cast<const uint32_t *>(src + 4);
        } else {
          const int8_t *rp = sigma + row * N;
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const int i = col + k < N ? col + k : N - 1;
            const uint32_t x = col + k < N ? uint32_t(uint8_t(rp[i])) : 0u;
            if (k < 4) a |= x << (8 * k);
            else b |= x << (8 * (k - 4));
          }
        }
      }
      *reinterpret_cast<uint4 *>(&sl[r * kRowW + 4 * (c < GPw ? c : WG)]) = spins8_bf16(a, b);
    }
    __syncthreads();
    if (vis) {
      // s_i from the sign bit of the staged bf16 spin, 8 sites per LDS read
      const int nw = N - c0 < 8 * GPw ? N - c0 : 8 * GPw;
      const uint32_t *sr = &sl[(64 * set + lane) * kRowW];
      for (int c = 0; c < GPw; ++c) {
        const uint4 d = *reinterpret_cast<const uint4 *>(sr + 4 * c);
        const uint32_t dw[4] = {d.x, d.y, d.z, d.w};
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int i = 8 * c + k;
          const uint32_t sb = dw[k >> 1] & ((k & 1) ? 0x80000000u : 0x8000u);
          const double x = i < nw ? (sb ? -1.0 : 1.0) : 0.0;
          const int ic = c0 + (i < nw ? i : nw - 1);
          vr += va[2 * ic] * x;
          vi += va[2 * ic + 1] * x;
        }
      }
    }
    if (active) {
      // step t: lane group hi takes k group 4 t + hi (part p of site group sg); the split
      // of step t + 1 is loaded while step t is contracted
      const int KSw = (3 * GPw + 3) / 4;
      const uint32_t *arow = &sl[(64 * set + lo) * kRowW];
      auto load_b = [&](int t, uint4 (&bv)[JT][PL]) {
        const int g8 = 4 * t + hi;
        const int sg = g8 / 3, p = g8 - 3 * sg;
        const int sgc = sg < GPw ? sg : GPw - 1;
        const uint32_t o = (uint32_t(p * GP + wg0 + sgc)) * uint32_t(M);
#pragma unroll
        for (int q = 0; q < JT; ++q)
#pragma unroll
          for (int pl = 0; pl < PL; ++pl) bv[q][pl] = Vs[o + jcl[q] + pl * plane];
      };
      auto step = [&](int t, const uint4 (&bv)[JT][PL]) {
        const int sg = (4 * t + hi) / 3;
        const uint32_t *ap = arow + 4 * (sg < GPw ? sg : WG);
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const uint4 av = *reinterpret_cast<const uint4 *>(ap + 16 * g * kRowW);
#pragma unroll
          for (int q = 0; q < JT; ++q)
#pragma unroll
            for (int pl = 0; pl < PL; ++pl)
              acc[g][q][pl] = mfma_bf16(av, bv[q][pl], acc[g][q][pl]);
        }
      };
      // two buffers in turn; a step past the last one reads the zero slot
      uint4 b0[JT][PL], b1[JT][PL];
      load_b(0, b0);
      for (int t = 0; t < KSw; t += 2) {
        load_b(t + 1 < KSw ? t + 1 : t, b1);
        step(t, b0);
        load_b(t + 2 < KSw ? t + 2 : t, b0);
        step(t + 1, b1);
      }
    }
  }
  if (!active) return;
  V<float, C> vbj[JT];
#pragma unroll
  for (int q = 0; q < JT; ++q) {
    const int j = (chunk * JT + q) * 16 + lo;
    vbj[q] = j < M ? vload<float, C>(vb, j) : vmake<float, C>(0.f, 0.f);
  }
  // T entries one group ahead of the group being summed
  auto load_t = [&](int g, V<float, C> (&tv)[JT][4]) {
#pragma unroll
    for (int q = 0; q < JT; ++q) {
      const int j = (chunk * JT + q) * 16 + lo;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = s0 + 16 * g + 4 * hi + r;
        const bool ok = j < M && row < n;
        const V<float, C> x = tload<float, C, TB>(Tm, ok ? row * M + j : 0);
        tv[q][r] = ok ? x : vmake<float, C>(0.f, 0.f);
      }
    }
  };
  V<float, C> tc[JT][4], tn[JT][4];
  load_t(0, tc);
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    if (g + 1 < 4) load_t(g + 1, tn);
    __builtin_amdgcn_sched_barrier(0);
    V<float, C> yp[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) yp[r] = vmake<float, C>(0.f, 0.f);
#pragma unroll
    for (int q = 0; q < JT; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const V<float, C> x = vmake<float, C>(acc[g][q][0][r] + vbj[q].re,
                                              C ? acc[g][q][C ? 1 : 0][r] + vbj[q].im : 0.f);
        yp[r] = vadd(yp[r], vmul(tc[q][r], x));
      }
    // sums over the 16 columns of each row; lane lo < 4 keeps row 4 hi + lo of the group
    float yr = 0.f, yi = 0.f;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float a = yp[r].re;
      a += dpp_f<DPP_QP_XOR1>(a);
      a += dpp_f<DPP_QP_XOR2>(a);
      a += dpp_f<DPP_ROR4>(a);
      a += dpp_f<DPP_ROR8>(a);
      yr = lo == r ? a : yr;
      if constexpr (C) {
        float b = yp[r].im;
        b += dpp_f<DPP_QP_XOR1>(b);
        b += dpp_f<DPP_QP_XOR2>(b);
        b += dpp_f<DPP_ROR4>(b);
        b += dpp_f<DPP_ROR8>(b);
        yi = lo == r ? b : yi;
      }
    }
    if (lo < 4) ysh[wid][16 * g + 4 * hi + lo] = make_double2(double(yr), double(yi));
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < JT; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) tc[q][r] = tn[q][r];
  }
  wave_sync();
  const int64_t s = s0 + lane;
  if (s < n) {
    const double2 y = ysh[wid][lane];
    *reinterpret_cast<double2 *>(ypart + 2 * (int64_t(chunk) * n + s)) =
        make_double2(y.x + vr, y.y + vi);
  }
}

template <bool C, bool TB>
__global__ __launch_bounds__(256, 2) void k_jvp32(int CW, int jchunks, int N, int M, int64_t n,
                                                   const int8_t *__restrict__ sigma,
                                                   const float *__restrict__ Tm,
                                                   const float *__restrict__ Vt,
                                                   const float *__restrict__ vb,
                                                   const double *__restrict__ va,
                                                   double *ypart, const int *skip) {
  k_jvp32_body<C, TB>(blockIdx.x, blockIdx.y, CW, jchunks, N, M, n, sigma, Tm, Vt, vb, va,
                      ypart, skip);
}

template <typename T, bool C>
__global__ __launch_bounds__(256) void k_jvp(int N, int M, int64_t n,
                                              const int8_t *__restrict__ sigma,
                                              const T *__restrict__ Tm,
                                              const T *__restrict__ Vt, const T *__restrict__ vb,
                                              const double *__restrict__ va, double *ypart,
                                              const int *skip) {
  k_jvp_body<T, C>(blockIdx.x, blockIdx.y, 0, 0, N, M, n, sigma, Tm, Vt, vb, va, ypart, skip);
}

// y[s] = sum over chunks; per-block partial sums of y (complex double) for centering
template <bool C>
__device__ __forceinline__ void k_jvp_finish_body(int BX, int BY, int BZ, int GX, int64_t n, int jchunks,
                                                     const double *__restrict__ ypart,
                                                     double *y, double *ysum_part,
                                                     const int *skip) {
  if (skip && *skip) return;
  __shared__ double sr[256], si[256];
  const int64_t s = int64_t(BX) * 256 + threadIdx.x;
  double yr = 0.0, yi = 0.0;
  if (s < n) {
    for (int c = 0; c < jchunks; ++c) {
      yr += ypart[2 * (int64_t(c) * n + s)];
      yi += ypart[2 * (int64_t(c) * n + s) + 1];
    }
    if (C) {
      y[2 * s] = yr;
      y[2 * s + 1] = yi;
    } else {
      y[s] = yr;
    }
  }
  if (ysum_part) {
    sr[threadIdx.x] = yr;
    si[threadIdx.x] = yi;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (int(threadIdx.x) < w) {
        sr[threadIdx.x] += sr[threadIdx.x + w];
        si[threadIdx.x] += si[threadIdx.x + w];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      ysum_part[2 * BX] = sr[0];
      ysum_part[2 * BX + 1] = si[0];
    }
  }
}

template <bool C>
__global__ __launch_bounds__(256) void k_jvp_finish(int64_t n, int jchunks,
                                                     const double *__restrict__ ypart,
                                                     double *y, double *ysum_part,
                                                     const int *skip) {
  k_jvp_finish_body<C>(blockIdx.x, blockIdx.y, blockIdx.z, gridDim.x, n, jchunks, ypart, y, ysum_part, skip);
}

// ---------------------------------------------------------------------------------
// VJP with stored T: G = Z^T S~ over a sample split, with rows j <= M and columns
// i <= N of the augmented operands
//   Z_sj = conj(T_sj) u_s (j < M),  Z_sM = u_s;   S~_si = s_si (i < N),  S~_sN = 1,
// so G[j][i] = (O^dagger u)_W_ji, G[j][N] = (O^dagger u)_b_j, G[M][i] = (O^dagger u)_a_i.
// A = Z^T needs no transpose: lane (lo, hi) loads Z[s + hi][j0 + lo]. Each wavefront
// accumulates JT x NT output tiles over every fourth 4-sample step of the block's split;
// the four wavefronts are summed through LDS and the block writes one partial tile set.
// Grid (hidden chunks, sample splits, site chunks).
// partial layout [split][Jtiles*16][Itiles*16], compute precision.
// ---------------------------------------------------------------------------------
// one 16-sample group of the FP32 VJP as loaded: u, the spins of the lane's site columns
// and the T entries of its hidden rows, for samples s + 4 hi + q (rows past send read row
// send - 1 with u = 0)
template <typename T, bool C, int JT, int NT>
struct VjpGroup {
  V<T, C> uu[4];
  int8_t sp[NT][4];
  V<T, C> tv[JT][4];
};
template <typename T, bool C, int JT, int NT, bool TB>
__device__ __forceinline__ void vjp_group_load(VjpGroup<T, C, JT, NT> &g,
                                               const int8_t *__restrict__ sigma,
                                               const T *__restrict__ Tm,
                                               const double *__restrict__ u, int N, int M,
                                               int64_t s, int64_t send, int hi, int lo, int jt0,
                                               int it0) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t row = s + 4 * hi + q;
    const bool ok = row < send;
    const int64_t rc = ok ? row : send - 1;
    const V<T, C> x = vmake<T, C>(T(u[C ? 2 * rc : rc]), C ? T(u[2 * rc + 1]) : T(0));
    g.uu[q] = ok ? x : vmake<T, C>(T(0), T(0));
#pragma unroll
    for (int b = 0; b < NT; ++b) {
      const int i = (it0 + b) * 16 + lo;
      g.sp[b][q] = sigma[rc * N + (i < N ? i : 0)];
    }
#pragma unroll
    for (int a = 0; a < JT; ++a) {
      const int j = (jt0 + a) * 16 + lo;
      g.tv[a][q] = tload<T, C, TB>(Tm, rc * M + (j < M ? j : 0));
    }
  }
}

template <typename T, bool C, int JT, int NT, bool TB = false>
__device__ __forceinline__ void k_vjp_body(int BX, int BY, int BZ, int GX, int N, int M, int64_t n,
                                              const int8_t *__restrict__ sigma,
                                              const T *__restrict__ Tm,
                                              const double *__restrict__ u, int64_t per_split,
                                              int rowsP, int colsP, T *part, const int *skip) {
  if (skip && *skip) return;
  typedef typename MF<T>::acc Acc;
  __shared__ T red[4][4][64][C ? 2 : 1];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int lo = lane & 15, hi = lane >> 4;
  const int jt0 = BX * JT, it0 = BZ * NT;
  const int64_t sbeg = int64_t(BY) * per_split;
  const int64_t send = sbeg + per_split < n ? sbeg + per_split : n;
  Acc ar[JT][NT], ai[JT][NT];
#pragma unroll
  for (int a = 0; a < JT; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) {
      ar[a][b] = Acc{0, 0, 0, 0};
      ai[a][b] = Acc{0, 0, 0, 0};
    }
  if constexpr (sizeof(T) == 4) {
    // FP32: 16-sample groups on the bf16 matrix cores. Lane (lo, hi) holds Z at samples
    // 4 hi + q (q < 4) of hidden row lo of each tile, split exactly into three bf16
    // parts (step 1: parts h and m, step 2: part l with a zero half) against the spins
    // of the same samples, which are exact in bf16. The next group's u, spins and T
    // entries are loaded while the current group is contracted (rows past the end of the
    // split read its last row and get u = 0, so their Z vanishes).
    VjpGroup<T, C, JT, NT> cur, nxt;
    const int64_t s0 = sbeg + 16 * wid;
    if (s0 < send)
      vjp_group_load<T, C, JT, NT, TB>(cur, sigma, Tm, u, N, M, s0, send, hi, lo, jt0, it0);
    for (int64_t s = s0; s < send; s += 64) {
      vjp_group_load<T, C, JT, NT, TB>(nxt, sigma, Tm, u, N, M, s + 64, send, hi, lo, jt0, it0);
      uint4 sb[NT];
#pragma unroll
      for (int b = 0; b < NT; ++b) {
        const int i = (it0 + b) * 16 + lo;
        T bs[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
          bs[q] = i < N ? T(cur.sp[b][q]) : (i == N ? T(1) : T(0));
        const uint32_t s01 = pack_hi(bs[0], bs[1]), s23 = pack_hi(bs[2], bs[3]);
        sb[b] = make_uint4(s01, s23, s01, s23);
      }
#pragma unroll
      for (int a = 0; a < JT; ++a) {
        const int j = (jt0 + a) * 16 + lo;
        V<T, C> z[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
          z[q] = j < M ? vmul(vconj(cur.tv[a][q]), cur.uu[q])
                       : (j == M ? cur.uu[q] : vmake<T, C>(T(0), T(0)));
#pragma unroll
        for (int pl = 0; pl < (C ? 2 : 1); ++pl) {
          T zz[4], r[4], l[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            zz[q] = pl ? z[q].im : z[q].re;
            r[q] = bf16_rest(zz[q]);
            l[q] = bf16_rest(r[q]);
          }
          const uint4 a0 = make_uint4(pack_hi(zz[0], zz[1]), pack_hi(zz[2], zz[3]),
                                      pack_hi(r[0], r[1]), pack_hi(r[2], r[3]));
          const uint4 a1 = make_uint4(pack_hi(l[0], l[1]), pack_hi(l[2], l[3]), 0u, 0u);
#pragma unroll
          for (int b = 0; b < NT; ++b) {
            if (pl) {
              ai[a][b] = mfma_bf16(a0, sb[b], ai[a][b]);
              ai[a][b] = mfma_bf16(a1, sb[b], ai[a][b]);
            } else {
              ar[a][b] = mfma_bf16(a0, sb[b], ar[a][b]);
              ar[a][b] = mfma_bf16(a1, sb[b], ar[a][b]);
            }
          }
        }
      }
      cur = nxt;
    }
  } else
  for (int64_t s = sbeg + 4 * wid; s < send; s += 16) {
    const int64_t srow = s + hi;
    const bool sok = srow < send;
    V<T, C> uu = vmake<T, C>(T(0), T(0));
    if (sok) uu = vmake<T, C>(T(u[C ? 2 * srow : srow]), C ? T(u[2 * srow + 1]) : T(0));
    V<T, C> z[JT];
#pragma unroll
    for (int a = 0; a < JT; ++a) {
      const int j = (jt0 + a) * 16 + lo;
      if (sok && j < M)
        z[a] = vmul(vconj(tload<T, C, TB>(Tm, srow * M + j)), uu);
      else
        z[a] = (sok && j == M) ? uu : vmake<T, C>(T(0), T(0));
    }
    T bs[NT];
    const int8_t *sp = sigma + (sok ? srow : 0) * N;
#pragma unroll
    for (int b = 0; b < NT; ++b) {
      const int i = (it0 + b) * 16 + lo;
      bs[b] = sok ? (i < N ? T(sp[i]) : (i == N ? T(1) : T(0))) : T(0);
    }
#pragma unroll
    for (int a = 0; a < JT; ++a)
#pragma unroll
      for (int b = 0; b < NT; ++b) {
        ar[a][b] = MF<T>::mma(z[a].re, bs[b], ar[a][b]);
        if constexpr (C) ai[a][b] = MF<T>::mma(z[a].im, bs[b], ai[a][b]);
      }
  }
  const int tid = threadIdx.x;
  const int r = tid >> 6, l = tid & 63;
#pragma unroll
  for (int a = 0; a < JT; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) {
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        red[wid][q][lane][0] = ar[a][b][q];
        if constexpr (C) red[wid][q][lane][C ? 1 : 0] = ai[a][b][q];
      }
      __syncthreads();
      const int jrow = (jt0 + a) * 16 + MF<T>::row(l >> 4, r);
      const int icol = (it0 + b) * 16 + (l & 15);
      if (jrow < rowsP && icol < colsP) {
        const int64_t o = (int64_t(BY) * rowsP + jrow) * colsP + icol;
        T sr = red[0][r][l][0] + red[1][r][l][0] + red[2][r][l][0] + red[3][r][l][0];
        if constexpr (C) {
          T si = red[0][r][l][C ? 1 : 0] + red[1][r][l][C ? 1 : 0] + red[2][r][l][C ? 1 : 0] +
                 red[3][r][l][C ? 1 : 0];
          part[2 * o] = sr;
          part[2 * o + 1] = si;
        } else {
          part[o] = sr;
        }
      }
    }
}

// Blocks of a launch are dispatched to the 8 XCDs of the device round-robin (block L to
// XCD L % 8, as that XCD's (L / 8)-th block), and every XCD has its own L2. The blocks of
// the site tiles (z) that read the same T rows (hidden tiles x, sample split y) are given
// consecutive slots on one XCD, so that the rows come from HBM once and from that XCD's L2
// for the other site tiles.
constexpr int kXcds = 8;

template <typename T, bool C, int JT, int NT, bool TB>
__global__ __launch_bounds__(256) void k_vjp(int gx, int gz, int64_t total, int N, int M,
                                              int64_t n, const int8_t *__restrict__ sigma,
                                              const T *__restrict__ Tm,
                                              const double *__restrict__ u, int64_t per_split,
                                              int rowsP, int colsP, T *part, const int *skip) {
  const int64_t per = (total + kXcds - 1) / kXcds;
  const int64_t L = blockIdx.x;
  const int64_t lam = (L % kXcds) * per + L / kXcds;
  if (lam >= total) return;
  const int bz = int(lam % gz);
  const int64_t rest = lam / gz;
  k_vjp_body<T, C, JT, NT, TB>(int(rest % gx), int(rest / gx), bz, gx, N, M, n, sigma, Tm, u,
                               per_split, rowsP, colsP, part, skip);
}

// ---------------------------------------------------------------------------------
// O^dagger u for FP32 / BF16 models whose site tiles all fit one block (5 to 17 tiles of 16
// sites): each block covers JT hidden tiles x every site tile over its sample split, so
// the exact bf16 split of Z = conj(T) u is formed once per element (not once per site-tile
// block). The spin operand comes from a table of bf16 quads written once per SR step
// (k_sigma_quads): sq[g][i] holds the spins of samples 4g .. 4g + 3 at site column i (1 in
// the bias column i = N, 0 past it and for samples past n), which is the MFMA's B operand
// of a lane as loaded. Two blocks per compute unit.
// sq[g][i] = 4 bf16 (samples 4g + q, q = 0..3, in the order of the lane's B operand)
__global__ void k_sigma_quads(int N, int cols, int64_t n, int64_t groups,
                              const int8_t *__restrict__ sigma, uint2 *__restrict__ sq) {
  const int64_t total = groups * cols;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t g = e / cols;
    const int i = int(e % cols);
    float v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t row = 4 * g + q;
      v[q] = row >= n ? 0.f : (i < N ? float(sigma[row * N + i]) : (i == N ? 1.f : 0.f));
    }
    sq[e] = make_uint2(pack_hi(v[0], v[1]), pack_hi(v[2], v[3]));
  }
}

template <bool C, int JT, int NT, bool TB>
__global__ __launch_bounds__(256, 2) void k_vjp_wide(int gx, int nt, int M, int64_t n,
                                                     const uint2 *__restrict__ sq, int cols,
                                                     const float *__restrict__ Tm,
                                                     const double *__restrict__ u,
                                                     int64_t per_split, int rowsP, float *part,
                                                     const int *skip) {
  if (skip && *skip) return;
  typedef floatx4 Acc;
  __shared__ float red[4][4][64][C ? 2 : 1];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int lo = lane & 15, hi = lane >> 4;
  const int bx = int(blockIdx.x % unsigned(gx)), by = int(blockIdx.x / unsigned(gx));
  const int jt0 = bx * JT;
  const int64_t sbeg = int64_t(by) * per_split;
  const int64_t send = sbeg + per_split < n ? sbeg + per_split : n;
  Acc ar[JT][NT], ai[JT][NT];
#pragma unroll
  for (int a = 0; a < JT; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) {
      ar[a][b] = Acc{0, 0, 0, 0};
      ai[a][b] = Acc{0, 0, 0, 0};
    }
  for (int64_t s = sbeg + 16 * wid; s < send; s += 64) {
    V<float, C> uu[4], tv[JT][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t row = s + 4 * hi + q;
      const bool ok = row < send;
      const int64_t rc = ok ? row : send - 1;
      const V<float, C> x =
          vmake<float, C>(float(u[C ? 2 * rc : rc]), C ? float(u[2 * rc + 1]) : 0.f);
      uu[q] = ok ? x : vmake<float, C>(0.f, 0.f);
#pragma unroll
      for (int a = 0; a < JT; ++a) {
        const int j = (jt0 + a) * 16 + lo;
        tv[a][q] = tload<float, C, TB>(Tm, rc * M + (j < M ? j : 0));
      }
    }
    const uint2 *sqg = sq + ((s + 4 * hi) >> 2) * int64_t(cols) + lo;
    uint4 sb[NT];
#pragma unroll
    for (int b = 0; b < NT; ++b) {
      if (b < nt) {
        const uint2 w = sqg[16 * b];
        sb[b] = make_uint4(w.x, w.y, w.x, w.y);
      }
    }
#pragma unroll
    for (int a = 0; a < JT; ++a) {
      const int j = (jt0 + a) * 16 + lo;
      V<float, C> z[4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        z[q] = j < M ? vmul(vconj(tv[a][q]), uu[q])
                     : (j == M ? uu[q] : vmake<float, C>(0.f, 0.f));
#pragma unroll
      for (int pl = 0; pl < (C ? 2 : 1); ++pl) {
        float zz[4], r[4], l[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          zz[q] = pl ? z[q].im : z[q].re;
          r[q] = bf16_rest(zz[q]);
          l[q] = bf16_rest(r[q]);
        }
        const uint4 a0 = make_uint4(pack_hi(zz[0], zz[1]), pack_hi(zz[2], zz[3]),
                                    pack_hi(r[0], r[1]), pack_hi(r[2], r[3]));
        const uint4 a1 = make_uint4(pack_hi(l[0], l[1]), pack_hi(l[2], l[3]), 0u, 0u);
#pragma unroll
        for (int b = 0; b < NT; ++b) {
          if (b < nt) {
            if (pl) {
              ai[a][b] = mfma_bf16(a0, sb[b], ai[a][b]);
              ai[a][b] = mfma_bf16(a1, sb[b], ai[a][b]);
            } else {
              ar[a][b] = mfma_bf16(a0, sb[b], ar[a][b]);
              ar[a][b] = mfma_bf16(a1, sb[b], ar[a][b]);
            }
          }
        }
      }
    }
  }
  const int tid = threadIdx.x;
  const int r = tid >> 6, l = tid & 63;
  const int colsP = cols;
#pragma unroll
  for (int a = 0; a < JT; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) {
      if (b >= nt) continue;
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        red[wid][q][lane][0] = ar[a][b][q];
        if constexpr (C) red[wid][q][lane][C ? 1 : 0] = ai[a][b][q];
      }
      __syncthreads();
      const int jrow = (jt0 + a) * 16 + MF<float>::row(l >> 4, r);
      const int icol = b * 16 + (l & 15);
      if (jrow < rowsP) {
        const int64_t o = (int64_t(by) * rowsP + jrow) * colsP + icol;
        const float sr = red[0][r][l][0] + red[1][r][l][0] + red[2][r][l][0] + red[3][r][l][0];
        if constexpr (C) {
          const float si = red[0][r][l][C ? 1 : 0] + red[1][r][l][C ? 1 : 0] +
                           red[2][r][l][C ? 1 : 0] + red[3][r][l][C ? 1 : 0];
          part[2 * o] = sr;
          part[2 * o + 1] = si;
        } else {
          part[o] = sr;
        }
      }
    }
}

// sum over the 16 lanes of each DPP row (every lane of the row receives the total)
template <typename T>
__device__ __forceinline__ T rowsum16(T x) {
  x += dpp_v<DPP_QP_XOR1>(x);
  x += dpp_v<DPP_QP_XOR2>(x);
  x += dpp_v<DPP_ROR4>(x);
  x += dpp_v<DPP_ROR8>(x);
  return x;
}

// ---------------------------------------------------------------------------------
// Fused S v product for shapes whose whole VJP output fits one block's tiles
// (ceil((M+1)/16) <= JT and ceil((N+1)/16) <= NT). Per 16-sample group a wavefront
//   1. forms y_s = sum_j T_sj (vb_j + (S V^T)_sj) + sum_i s_si va_i (X by MFMA, the
//      hidden-unit sum by DPP row reductions),
//   2. accumulates O^dagger y with Z_sj = conj(T_sj) y_s over the same samples, while
//      their T rows are still in cache,
// so T is streamed from memory once per product. Output: one partial tile set per
// block (as k_vjp) and the block's sum of y (complex double) for the centring.
// Grid: sample splits. Vt is staged in LDS when VL.
// ---------------------------------------------------------------------------------
template <typename T, bool C, int JT, int NT>
__global__ __launch_bounds__(256) void k_sv(int N, int M, int64_t n,
                                             const int8_t *__restrict__ sigma,
                                             const T *__restrict__ Tm, const T *__restrict__ Vt_g,
                                             const T *__restrict__ vb,
                                             const double *__restrict__ va, int64_t per_split,
                                             int rowsP, int colsP, T *part, double *ysum_part,
                                             const int *skip) {
  if (skip && *skip) return;
  typedef typename MF<T>::acc Acc;
  constexpr int cs = C ? 2 : 1;
  constexpr int JW = JT * 16;  // padded hidden width of the staged direction
  constexpr int SW = NT * 16;  // padded site width of the spin tile (>= N + 1)
  extern __shared__ __align__(16) unsigned char lds_u8[];
  __shared__ T red[4][4][64][cs];
  __shared__ double dsum[2][256];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int lo = lane & 15, hi = lane >> 4;
  const int Kp = (N + 3) / 4 * 4;
  // dynamic LDS: V^T zero-padded to [Kp][JW], then one 16 x SW spin tile per wavefront
  T *Vl = reinterpret_cast<T *>(lds_u8);
  const int64_t vbytes = (int64_t(Kp) * JW * cs * int64_t(sizeof(T)) + 15) / 16 * 16;
  int8_t *stile = reinterpret_cast<int8_t *>(lds_u8 + vbytes) + wid * 16 * SW;
  for (int e = threadIdx.x; e < Kp * JW; e += 256) {
    const int k = e / JW, j = e % JW;
    const V<T, C> v = (k < N && j < M) ? vload<T, C>(Vt_g, int64_t(k) * M + j)
                                       : vmake<T, C>(T(0), T(0));
    vstore<T, C>(Vl, e, v);
  }
  __syncthreads();
  const int64_t sbeg = int64_t(blockIdx.x) * per_split;
  const int64_t send = sbeg + per_split < n ? sbeg + per_split : n;
  Acc ar[JT][NT], ai[JT][NT];
#pragma unroll
  for (int a = 0; a < JT; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) {
      ar[a][b] = Acc{0, 0, 0, 0};
      ai[a][b] = Acc{0, 0, 0, 0};
    }
  double ysr = 0.0, ysi = 0.0;
  const int Mt = (M + 15) / 16;
  // spin-tile fill: lane owns row lane/4 and columns lane%4 + 4 c
  const int frow = lane >> 2, fcol = lane & 3;
  for (int64_t g = sbeg + 16 * wid; g < send; g += 64) {
    const int rows_here = send - g < 16 ? int(send - g) : 16;
    // T tile of the group in the accumulator layout: lane (lo, hi) holds rows
    // MF::row(hi, r), columns 16 a + lo. The same registers feed the JVP epilogue and,
    // with the VJP samples of step q taken as row MF::row(hi, q), the VJP A operand.
    V<T, C> tv[JT][4];
#pragma unroll
    for (int a = 0; a < JT; ++a) {
      const int j = a * 16 + lo;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = MF<T>::row(hi, r);
        tv[a][r] = (a < Mt && j < M && rr < rows_here) ? vload<T, C>(Tm, (g + rr) * M + j)
                                                       : vmake<T, C>(T(0), T(0));
      }
    }
    // spins of the 16 samples, zero-padded, with a column of ones at site N (hidden bias)
    wave_sync();
    {
      const bool rok = frow < rows_here;
      const int8_t *src = sigma + (g + (rok ? frow : 0)) * N;
      for (int c = fcol; c < SW; c += 4) {
        int8_t v = 0;
        if (rok) v = c < N ? src[c] : (c == N ? int8_t(1) : int8_t(0));
        stile[frow * SW + c] = v;
      }
    }
    wave_sync();
    // ---- y for rows g .. g+15: X = S V^T for all hidden tiles, A operand loaded once ----
    Acc xr[JT], xi[JT];
#pragma unroll
    for (int a = 0; a < JT; ++a) {
      xr[a] = Acc{0, 0, 0, 0};
      xi[a] = Acc{0, 0, 0, 0};
    }
    for (int k0 = 0; k0 < Kp; k0 += 4) {
      const int k = k0 + hi;
      const T av = T(stile[lo * SW + k]);
      V<T, C> v[JT];
#pragma unroll
      for (int a = 0; a < JT; ++a) v[a] = vload<T, C>(Vl, int64_t(k) * JW + a * 16 + lo);
#pragma unroll
      for (int a = 0; a < JT; ++a) {
        xr[a] = MF<T>::mma(av, v[a].re, xr[a]);
        if constexpr (C) xi[a] = MF<T>::mma(av, v[a].im, xi[a]);
      }
    }
    V<T, C> yp[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) yp[r] = vmake<T, C>(T(0), T(0));
#pragma unroll
    for (int a = 0; a < JT; ++a) {
      const int j = a * 16 + lo;
      const V<T, C> vbj = (a < Mt && j < M) ? vload<T, C>(vb, j) : vmake<T, C>(T(0), T(0));
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        V<T, C> x = vmake<T, C>(xr[a][r] + vbj.re, C ? xi[a][r] + vbj.im : T(0));
        yp[r] = vadd(yp[r], vmul(tv[a][r], x));
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int rr = MF<T>::row(hi, r);
      for (int i = lo; i < N; i += 16) {
        const T si = T(stile[rr * SW + i]);
        yp[r].re += si * T(va[2 * i]);
        if constexpr (C) yp[r].im += si * T(va[2 * i + 1]);
      }
      yp[r].re = rowsum16(yp[r].re);
      if constexpr (C) yp[r].im = rowsum16(yp[r].im);
      if (rr >= rows_here) yp[r] = vmake<T, C>(T(0), T(0));
      if (lo == 0) {
        ysr += double(yp[r].re);
        if constexpr (C) ysi += double(yp[r].im);
      }
    }
    // ---- accumulate O^dagger y over the same 16 samples (step q: row MF::row(hi, q)) ----
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int rr = MF<T>::row(hi, q);
      V<T, C> z[JT];
#pragma unroll
      for (int a = 0; a < JT; ++a) {
        const int j = a * 16 + lo;
        z[a] = j < M ? vmul(vconj(tv[a][q]), yp[q])
                     : (j == M ? yp[q] : vmake<T, C>(T(0), T(0)));
      }
      T bs[NT];
#pragma unroll
      for (int b = 0; b < NT; ++b) bs[b] = T(stile[rr * SW + b * 16 + lo]);
#pragma unroll
      for (int a = 0; a < JT; ++a)
#pragma unroll
        for (int b = 0; b < NT; ++b) {
          ar[a][b] = MF<T>::mma(z[a].re, bs[b], ar[a][b]);
          if constexpr (C) ai[a][b] = MF<T>::mma(z[a].im, bs[b], ai[a][b]);
        }
    }
  }
  // block sums: partial tiles, then sum of y
  const int tid = threadIdx.x;
  const int r = tid >> 6, l = tid & 63;
#pragma unroll
  for (int a = 0; a < JT; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) {
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        red[wid][q][lane][0] = ar[a][b][q];
        if constexpr (C) red[wid][q][lane][cs - 1] = ai[a][b][q];
      }
      __syncthreads();
      const int jrow = a * 16 + MF<T>::row(l >> 4, r);
      const int icol = b * 16 + (l & 15);
      if (jrow < rowsP && icol < colsP) {
        const int64_t o = (int64_t(blockIdx.x) * rowsP + jrow) * colsP + icol;
        T sr = red[0][r][l][0] + red[1][r][l][0] + red[2][r][l][0] + red[3][r][l][0];
        if constexpr (C) {
          T si = red[0][r][l][cs - 1] + red[1][r][l][cs - 1] + red[2][r][l][cs - 1] +
                 red[3][r][l][cs - 1];
          part[2 * o] = sr;
          part[2 * o + 1] = si;
        } else {
          part[o] = sr;
        }
      }
    }
  dsum[0][tid] = ysr;
  dsum[1][tid] = ysi;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) {
      dsum[0][tid] += dsum[0][tid + w];
      dsum[1][tid] += dsum[1][tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) {
    ysum_part[2 * blockIdx.x] = dsum[0][0];
    ysum_part[2 * blockIdx.x + 1] = dsum[1][0];
  }
}

// Spins of every sample as a 64-bit mask (bit i set when spin i is up), N <= 63.
__global__ void k_pack_spins(int N, int64_t n, const int8_t *__restrict__ sigma,
                             uint64_t *masks) {
  const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int8_t *row = sigma + s * N;
  uint64_t m = 0;
  for (int i = 0; i < N; ++i) m |= uint64_t(row[i] > 0) << i;
  masks[s] = m;
}

// rows of the 16-sample group starting at g that lie before send (0..16)
__device__ __forceinline__ int svc_rows(int64_t send, int64_t g) {
  const int64_t left = send - g;
  return left <= 0 ? 0 : (left < 16 ? int(left) : 16);
}

// the spin masks of rows 4 hi + q (mq[q]) and lane % 16 (mlo) and the T rows of one
// 16-sample group (rows 4 hi + r, hidden tiles below JV). One code path for every group:
// rows past the last valid one (rows_here of them, 0 past the end of the split) read the
// last valid row instead, and their y is zeroed later, so their Z = conj(T) y vanishes
// exactly; columns j >= M of the last tile read the next row (or the slack after T) and
// meet zero direction entries in the JVP and ignored output rows in the VJP. Addresses
// are a uniform row base plus a 32-bit lane offset.
template <typename T, int JT, int JV, bool TB>
__device__ __forceinline__ void svc_load(const uint64_t *__restrict__ masks,
                                         const T *__restrict__ Tm, int M, int64_t g,
                                         int64_t send, int rows_here, int lane, int lo, int hi,
                                         uint64_t (&mq)[4], uint64_t &mlo,
                                         V<T, true> (&tv)[JT][4]) {
  const int64_t gb = rows_here > 0 ? g : send - 1;
  const int rmax = rows_here > 0 ? rows_here - 1 : 0;
  const uint64_t *mb = masks + gb;
#pragma unroll
  for (int q = 0; q < 4; ++q) mq[q] = mb[min(4 * hi + q, rmax)];
  mlo = mb[min(lo, rmax)];
  // (complex entries of 8 bytes, or 4 as bfloat16 pairs: one T unit per entry)
  const T *tb = Tm + (TB ? 1 : 2) * gb * int64_t(M);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const uint32_t off = uint32_t((TB ? 1 : 2) * (min(MF<T>::row(hi, r), rmax) * M + lo));
#pragma unroll
    for (int a = 0; a < JT; ++a)
      tv[a][r] = a < JV ? tload<T, true, TB>(tb + off, a * 16) : vmake<T, true>(T(0), T(0));
  }
}

// ---------------------------------------------------------------------------------
// Fused S v product for complex models with N <= 63 and all VJP tiles in one block.
// The real and imaginary planes of both contractions are split between the two
// wavefronts of a pair, which then hold half the accumulators each (two pairs = two
// 16-sample groups in flight per block, two blocks per SIMD). Wavefront h of a pair:
//   X_h = S (plane h of V)^T by MFMA, and its share of y:
//     h = 0: Re y += Re T (X_0 + Re vb) + s.Re va,  Im y += Im T (X_0 + Re vb) + s.Im va
//     h = 1: Re y -= Im T (X_1 + Im vb),            Im y += Re T (X_1 + Im vb)
//   the 16 partial sums of y are exchanged through LDS (double-buffered, flag-synchronised
//   within the pair);
//   then plane h of Z^T S with Z = conj(T) y:
//     Re Z = Re T Re y + Im T Im y,  Im Z = Re T Im y - Im T Re y  (row M: Z = y).
// Spins enter as 64-bit masks (k_pack_spins): the JVP operand through a byte table, the
// VJP operand and the visible term from the mask bits of each lane's four sample rows
// (4 hi + q, column lo + 16 c). Both contractions run on the bf16 matrix
// cores: the FP32 factor (V, then Z) is split exactly into three bf16 parts against the
// +/-1 spins, so the products are exact and the sums FP32.
// JT = ceil((M+1)/16) hidden tiles of the VJP output, JV = ceil(M/16) of them carry
// hidden units in the JVP, NT = ceil((N+1)/16) site tiles.
// ---------------------------------------------------------------------------------
// dynamic LDS of k_svc: the bf16 split of V for both planes ([2][G][16 JV] groups of
// 8 bf16, G = 4 ceil(3 ceil(N / 8) / 4), JV = ceil(M / 16))
inline size_t svc_dynamic_lds(int N, int M) {
  const size_t G = size_t(4) * ((3 * ((N + 7) / 8) + 3) / 4);
  const size_t JVW = size_t((M + 15) / 16) * 16;
  return 2 * G * JVW * 16;
}

template <typename T, int JT, int JV, int NT, int PAIRS, bool TB>
__global__ __launch_bounds__(128 * PAIRS, 2) void k_svc(int N, int M, int64_t n,
                                                const uint64_t *__restrict__ masks,
                                                const T *__restrict__ Tm,
                                                const T *__restrict__ Vt_g,
                                                const T *__restrict__ vb,
                                                const double *__restrict__ va,
                                                int64_t per_split, int rowsP, int colsP,
                                                T *part, double *ysum_part, const int *skip) {
  // a finished solve returns after the staging below (the flag is read with its loads)
  const int skipped = skip ? *skip : 0;
  typedef typename MF<T>::acc Acc;
  constexpr int JW = JT * 16;
  constexpr int NVA = 4;                        // site columns per lane: lo + 16 c, N <= 63
  static_assert(NT <= NVA, "site tiles of the VJP within the lane's spin columns");
  extern __shared__ __align__(16) unsigned char lds_u8[];
  static_assert(sizeof(T) == 4, "the bf16 split is FP32");
  constexpr int NTH = 128 * PAIRS;
  __shared__ T ybuf[2][PAIRS][2][16][2];  // [parity][pair][plane of origin][row][re, im]
  __shared__ T red[2 * PAIRS][4][64];
  __shared__ double dsum[2][2 * PAIRS];
  // spin byte b -> the 8 spins (bit e set: +1, else -1) as bf16, element e = site e
  __shared__ __align__(16) uint32_t stab[256 * 4];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int lo = lane & 15, hi = lane >> 4;
  const int pr = wid >> 1, h = wid & 1;
  // JVP contraction dimension: k group g (8 consecutive k) = part g % 3 of the bf16 split
  // of V at sites 8 (g / 3) .. 8 (g / 3) + 7; GP site groups, KS steps of 32 k, and
  // G = 4 KS groups per plane (those from 3 GP on are zero)
  const int GP = (N + 7) >> 3;
  const int KS = (3 * GP + 3) >> 2;
  const int G = 4 * KS;
  constexpr int JVW = JV * 16;
  uint4 *Vb = reinterpret_cast<uint4 *>(lds_u8);  // [plane][G][JVW]: B operands of the JVP
  for (int e = threadIdx.x; e < GP * JVW; e += NTH) {
    const int sg = e / JVW, j = e - sg * JVW;
    uint32_t w[2][3][4];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = 8 * sg + u;
      V<T, true> x = vmake<T, true>(T(0), T(0));
      if (i < N && j < M) x = vload<T, true>(Vt_g, int64_t(i) * M + j);
#pragma unroll
      for (int pl = 0; pl < 2; ++pl) {
        const float v0 = pl ? x.im : x.re;
        const float r = bf16_rest(v0), l = bf16_rest(r);
        const uint32_t bits[3] = {__float_as_uint(v0) >> 16, __float_as_uint(r) >> 16,
                                  __float_as_uint(l) >> 16};
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          if (u & 1)
            w[pl][q][u >> 1] |= bits[q] << 16;
          else
            w[pl][q][u >> 1] = bits[q];
        }
      }
    }
#pragma unroll
    for (int pl = 0; pl < 2; ++pl)
#pragma unroll
      for (int q = 0; q < 3; ++q)
        Vb[(pl * G + 3 * sg + q) * JVW + j] =
            make_uint4(w[pl][q][0], w[pl][q][1], w[pl][q][2], w[pl][q][3]);
  }
  {
    const int pad = G - 3 * GP;
    for (int e = threadIdx.x; e < 2 * pad * JVW; e += NTH) {
      const int q = e / JVW, j = e - q * JVW;
      const int pl = q / pad, gq = 3 * GP + (q - pl * pad);
      Vb[(pl * G + gq) * JVW + j] = make_uint4(0u, 0u, 0u, 0u);
    }
  }
  for (int e = threadIdx.x; e < 256 * 4; e += NTH) {
    const uint32_t b = uint32_t(e) >> 2, u = uint32_t(e) & 3u;
    const uint32_t s0 = ((b >> (2 * u)) & 1u) ? 0x3F80u : 0xBF80u;
    const uint32_t s1 = ((b >> (2 * u + 1)) & 1u) ? 0x3F80u : 0xBF80u;
    stab[e] = s0 | (s1 << 16);
  }
  // both planes of vb (zero past M) and va (zero past N) in LDS, read per group
  __shared__ T vbl[2][JW];
  __shared__ T val[2][16 * NVA];
  __shared__ int pflag[2 * PAIRS];  // per wavefront: groups whose partial y is published
  if (threadIdx.x < 2 * PAIRS) pflag[threadIdx.x] = 0;
  for (int e = threadIdx.x; e < 2 * JW; e += NTH) {
    const int pl = e / JW, j = e - pl * JW;
    vbl[pl][j] = j < M ? vb[2 * j + pl] : T(0);
  }
  for (int e = threadIdx.x; e < 2 * 16 * NVA; e += NTH) {
    const int pl = e / (16 * NVA), i = e - pl * (16 * NVA);
    val[pl][i] = i < N ? T(va[2 * i + pl]) : T(0);
  }
  __syncthreads();
  if (skipped) return;
  bool stalled = false;
  const int64_t sbeg = int64_t(blockIdx.x) * per_split;
  const int64_t send = sbeg + per_split < n ? sbeg + per_split : n;
  const int64_t iters = send > sbeg ? (send - sbeg + 16 * PAIRS - 1) / (16 * PAIRS) : 0;
  // row-M tile on the vector units when it holds nothing else (M a multiple of 16)
  constexpr bool AROW = JV == JT - 1;
  constexpr int JTM = AROW ? JT - 1 : JT;  // hidden tiles accumulated on the matrix cores
  Acc acc[JTM][NT];
#pragma unroll
  for (int a = 0; a < JTM; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) acc[a][b] = Acc{0, 0, 0, 0};
  T ga[NT];
#pragma unroll
  for (int b = 0; b < NT; ++b) ga[b] = T(0);
  double ysr = 0.0, ysi = 0.0;
  // per-lane constants of the group loop: the byte shift of the JVP A operand at each
  // step (k group 4 t + hi covers sites 8 ((4 t + hi) / 3) ..), the lane's bias entries
  constexpr int KSMAX = 6;  // N <= 63: 3 ceil(N / 8) <= 24 k groups
  uint32_t ash[KSMAX];
#pragma unroll
  for (int t = 0; t < KSMAX; ++t) ash[t] = uint32_t(8 * ((4 * t + hi) / 3));
  // the loop is specialised for the plane H of the wavefront (uniform branch below):
  // plane 1 uses i T = (-Im T, Re T), so that with (Re', Im') the plane's view of T
  //   y += (Re', Im') (X_H + vb_H),  Z_H = Re' Re y + Im' Im y
  auto run = [&](auto hc) __attribute__((always_inline)) {
    constexpr int H = decltype(hc)::value;
    T vbr[JV], var[NVA];
#pragma unroll
    for (int a = 0; a < JV; ++a) vbr[a] = vbl[H][a * 16 + lo];
#pragma unroll
    for (int c = 0; c < NVA; ++c) var[c] = val[H][lo + 16 * c];
    // spins as factors at column i = lo + 16 c of the sample rows: +/-1 from the mask bit
    // for i < N, 1 at i = N (the ones column of the bias gradients), 0 beyond (mask bits
    // are clear from N on)
    T shi[NVA], slo[NVA];
#pragma unroll
    for (int c = 0; c < NVA; ++c) {
      const int i = lo + 16 * c;
      shi[c] = i < N ? T(1) : T(0);
      slo[c] = i < N ? T(-1) : (i == N ? T(1) : T(0));
    }
    auto spin = [&](const uint64_t (&m)[4], int q, int c) __attribute__((always_inline)) -> T {
      const uint32_t w = c < 2 ? uint32_t(m[q]) : uint32_t(m[q] >> 32);
      return ((w >> (lo + 16 * (c & 1))) & 1u) ? shi[c] : slo[c];
    };
    const uint4 *tab4 = reinterpret_cast<const uint4 *>(stab);
    const uint4 *Vh = Vb + H * G * JVW + lo;
    // software pipeline: the masks and T rows of the pair's next group are loaded while
    // the current group's O^dagger y contraction runs
    int64_t g = sbeg + 16 * pr;
    int rows_here = svc_rows(send, g);
    uint64_t mq[4], mlo;
    V<T, true> tv[JT][4];
    if (iters > 0) svc_load<T, JT, JV, TB>(masks, Tm, M, g, send, rows_here, lane, lo, hi, mq, mlo, tv);
    for (int64_t it = 0; it < iters; ++it) {
      // the masks of rows 4 hi + q of this group (the loads below fetch the next group's)
      uint64_t mc[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) mc[q] = mq[q];
      // ---- X_H = S (plane H of V)^T over the valid hidden tiles, bf16 split ----
      // A (sample lo, k group g): the spins of sites 8 (g / 3) .. + 7 from the byte
      // table; sites past N meet zeros in B. Steps unrolled to KSMAX, uniform guards.
      Acc x[JV];
#pragma unroll
      for (int t = 0; t < KSMAX; ++t) {
        if (t < KS) {
          const uint4 av = tab4[uint32_t(mlo >> ash[t]) & 0xffu];
          uint4 bv[JV];
#pragma unroll
          for (int a = 0; a < JV; ++a) bv[a] = Vh[(4 * t + hi) * JVW + 16 * a];
#pragma unroll
          for (int a = 0; a < JV; ++a)
            x[a] = mfma_bf16(av, bv[a], t == 0 ? Acc{0, 0, 0, 0} : x[a]);
        }
      }
      // ---- this plane's share of y for rows MF::row(hi, r) ----
      T yre[4], yim[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        yre[r] = T(0);
        yim[r] = T(0);
      }
#pragma unroll
      for (int a = 0; a < JV; ++a) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const T xv = x[a][r] + vbr[a];
          if constexpr (H == 0) {
            yre[r] += tv[a][r].re * xv;
            yim[r] += tv[a][r].im * xv;
          } else {
            yre[r] -= tv[a][r].im * xv;
            yim[r] += tv[a][r].re * xv;
          }
        }
      }
      if constexpr (H == 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
#pragma unroll
          for (int c = 0; c < NVA; ++c) yre[r] += spin(mc, r, c) * var[c];  // va is 0 from N on
        }
      }
      if constexpr (H == 1) {
        // the imaginary part of va enters through plane 1's share of Im y
#pragma unroll
        for (int r = 0; r < 4; ++r) {
#pragma unroll
          for (int c = 0; c < NVA; ++c) yim[r] += spin(mc, r, c) * var[c];
        }
      }
      const int par = int(it & 1);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        yre[r] = rowsum16(yre[r]);
        yim[r] = rowsum16(yim[r]);
      }
      if (rows_here < 16) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (MF<T>::row(hi, r) >= rows_here) {
            yre[r] = T(0);
            yim[r] = T(0);
          }
      }
      if (lo == 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int rr = MF<T>::row(hi, r);
          ybuf[par][pr][H][rr][0] = yre[r];
          ybuf[par][pr][H][rr][1] = yim[r];
        }
      }
      // publish this wavefront's partial sums, then wait (bounded) for the partner's: the
      // two wavefronts of a pair synchronise through LDS flags only, so pairs drift apart
      // and one wavefront's VALU work overlaps the other's matrix-core work on a SIMD
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      if (lane == 0)
        __hip_atomic_store(&pflag[wid], int(it + 1), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
      {
        int spins = 0;
#pragma nounroll
        while (__builtin_amdgcn_readfirstlane(__hip_atomic_load(
                   &pflag[wid ^ 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) <
               int(it + 1)) {
          __builtin_amdgcn_s_sleep(1);
          if (++spins > (1 << 24)) {
            stalled = true;
            break;
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = MF<T>::row(hi, r);
        yre[r] += ybuf[par][pr][H ^ 1][rr][0];
        yim[r] += ybuf[par][pr][H ^ 1][rr][1];
      }
      if constexpr (H == 0) {
        if (lo == 0) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            ysr += double(yre[r]);
            ysi += double(yim[r]);
          }
        }
      }
      // ---- plane H of Z = conj(T) y (row M: Z = y), then the next group's loads ----
      T z[4][JTM];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int a = 0; a < JTM; ++a) {
          T zq;
          if constexpr (H == 0)
            zq = tv[a][q].re * yre[q] + tv[a][q].im * yim[q];
          else
            zq = tv[a][q].re * yim[q] - tv[a][q].im * yre[q];
          if constexpr (!AROW) {
            if (a == JT - 1 && a * 16 + lo == M) zq = H == 0 ? yre[q] : yim[q];
          }
          z[q][a] = zq;
        }
      }
      __builtin_amdgcn_sched_barrier(0);  // keep the next loads after the last reads of tv
      // unconditional (after the last group they re-read a valid row), so the loaded
      // registers are the next iteration's operands with no merge copies
      g += 16 * PAIRS;
      rows_here = svc_rows(send, g);
      svc_load<T, JT, JV, TB>(masks, Tm, M, g, send, rows_here, lane, lo, hi, mq, mlo, tv);
      // ---- plane H of Z^T S over the 16 samples, bf16 split of Z ----
      // k of lane group hi: element e < 4 pairs part h of Z at sample 4 hi + e with that
      // sample's spin, e >= 4 part m; a second step takes part l (upper half zero).
      // With M a multiple of 16 the last hidden tile holds only row M (Z = y): its sums
      // g_a = sum_s y_s s_s are accumulated on the vector units instead.
      uint4 sb[NT];
#pragma unroll
      for (int b = 0; b < NT; ++b) {
        T bs[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) bs[q] = spin(mc, q, b);
        if constexpr (AROW) {
#pragma unroll
          for (int q = 0; q < 4; ++q) ga[b] += (H == 0 ? yre[q] : yim[q]) * bs[q];
        }
        const uint32_t s01 = pack_hi(bs[0], bs[1]), s23 = pack_hi(bs[2], bs[3]);
        sb[b] = make_uint4(s01, s23, s01, s23);
      }
#pragma unroll
      for (int a = 0; a < JTM; ++a) {
        T r[4], l[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          r[q] = bf16_rest(z[q][a]);
          l[q] = bf16_rest(r[q]);
        }
        const uint4 a0 = make_uint4(pack_hi(z[0][a], z[1][a]), pack_hi(z[2][a], z[3][a]),
                                    pack_hi(r[0], r[1]), pack_hi(r[2], r[3]));
        const uint4 a1 = make_uint4(pack_hi(l[0], l[1]), pack_hi(l[2], l[3]), 0u, 0u);
#pragma unroll
        for (int b = 0; b < NT; ++b) acc[a][b] = mfma_bf16(a0, sb[b], acc[a][b]);
#pragma unroll
        for (int b = 0; b < NT; ++b) acc[a][b] = mfma_bf16(a1, sb[b], acc[a][b]);
      }
    }
  };
  if (h == 0)
    run(std::integral_constant<int, 0>{});
  else
    run(std::integral_constant<int, 1>{});
  if constexpr (AROW) {
    // lanes of one column (lo) hold the sums of rows 4 hi .. 4 hi + 3: add the four
#pragma unroll
    for (int b = 0; b < NT; ++b) {
      ga[b] += __shfl_xor(ga[b], 16, 64);
      ga[b] += __shfl_xor(ga[b], 32, 64);
    }
  }
  // block sums: plane 0 of every pair -> real part, plane 1 -> imaginary part
  const int tid = threadIdx.x;
  const int r = (tid >> 6) & 3, l = tid & 63;
#pragma unroll
  for (int a = 0; a < JT; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) {
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (a < JTM)
          red[wid][q][lane] = acc[a < JTM ? a : 0][b][q];
        else  // the row-M tile: only row M is nonzero
          red[wid][q][lane] = a * 16 + MF<T>::row(hi, q) == M ? ga[b] : T(0);
      }
      __syncthreads();
      const int jrow = a * 16 + MF<T>::row(l >> 4, r);
      const int icol = b * 16 + (l & 15);
      if (tid < 256 && jrow < rowsP && icol < colsP) {
        const int64_t o = (int64_t(blockIdx.x) * rowsP + jrow) * colsP + icol;
        T sr = T(0), si = T(0);
#pragma unroll
        for (int p = 0; p < PAIRS; ++p) {
          sr += red[2 * p][r][l];
          si += red[2 * p + 1][r][l];
        }
        part[2 * o] = sr;
        part[2 * o + 1] = si;
      }
    }
  // a wavefront that gave up waiting for its partner poisons the block's sum of y, so
  // the solver reports a non-finite result instead of a wrong one
  {
    // wavefront sums (DPP), then the wavefronts in index order
    const double wr = wave_sum_dpp(ysr), wi = wave_sum_dpp(ysi);
    if (lane == 0) {
      dsum[0][wid] = stalled ? __builtin_nan("") : wr;
      dsum[1][wid] = wi;
    }
    __syncthreads();
    if (tid == 0) {
      double sr = 0.0, si = 0.0;
      for (int w = 0; w < 2 * PAIRS; ++w) {
        sr += dsum[0][w];
        si += dsum[1][w];
      }
      ysum_part[2 * blockIdx.x] = sr;
      ysum_part[2 * blockIdx.x + 1] = si;
    }
  }
}

// first reduction level: out1[g][e] = sum of partials of split group g (complex double)
template <typename T, bool C>
__device__ __forceinline__ void k_vjp_reduce1_body(int BX, int BY, int BZ, int GX, int splits, int groups, int64_t elems,
                                                     const T *__restrict__ part, double *out1,
                                                     const int *skip) {
  if (skip && *skip) return;
  const int64_t e = int64_t(BX) * 256 + threadIdx.x;
  if (e >= elems) return;
  const int g = BY;
  const int per = (splits + groups - 1) / groups;
  const int p0 = g * per, p1 = p0 + per < splits ? p0 + per : splits;
  double sr = 0.0, si = 0.0;
  for (int p = p0; p < p1; ++p) {
    V<T, C> x = vload<T, C>(part, int64_t(p) * elems + e);
    sr += double(x.re);
    si += double(x.im);
  }
  out1[2 * (int64_t(g) * elems + e)] = sr;
  out1[2 * (int64_t(g) * elems + e) + 1] = si;
}

template <typename T, bool C>
__global__ __launch_bounds__(256) void k_vjp_reduce1(int splits, int groups, int64_t elems,
                                                     const T *__restrict__ part, double *out1,
                                                     const int *skip) {
  k_vjp_reduce1_body<T, C>(blockIdx.x, blockIdx.y, blockIdx.z, gridDim.x, splits, groups, elems, part, out1, skip);
}

// second level: out[k] (double, packed like the parameters) = sum over groups
template <bool C>
__device__ __forceinline__ void k_vjp_reduce2_body(int BX, int BY, int BZ, int GX, int N, int M, int groups, int colsP, int64_t elems,
                              const double *__restrict__ out1, double *out, const int *skip) {
  if (skip && *skip) return;
  const int64_t P = int64_t(N) + M + int64_t(N) * M;
  for (int64_t k = BX * int64_t(blockDim.x) + threadIdx.x; k < P;
       k += int64_t(GX) * blockDim.x) {
    int64_t e;
    if (k < N) {
      e = int64_t(M) * colsP + k;                 // row M: visible bias
    } else if (k < N + M) {
      e = int64_t(k - N) * colsP + N;             // column N: hidden bias
    } else {
      const int64_t q = k - N - M;
      e = (q / N) * colsP + (q % N);              // W_ji
    }
    double sr = 0.0, si = 0.0;
    for (int g = 0; g < groups; ++g) {
      sr += out1[2 * (int64_t(g) * elems + e)];
      si += out1[2 * (int64_t(g) * elems + e) + 1];
    }
    if (C) {
      out[2 * k] = sr;
      out[2 * k + 1] = si;
    } else {
      out[k] = sr;
    }
  }
}

template <bool C>
__global__ void k_vjp_reduce2(int N, int M, int groups, int colsP, int64_t elems,
                              const double *__restrict__ out1, double *out, const int *skip) {
  k_vjp_reduce2_body<C>(blockIdx.x, blockIdx.y, blockIdx.z, gridDim.x, N, M, groups, colsP, elems, out1, out, skip);
}

// ---------------------------------------------------------------------------------
// scratch layout (byte offsets), all regions 256-byte aligned
// ---------------------------------------------------------------------------------
struct GradLayout {
  size_t Vt, vb, va, ypart, Tm, masks, sq, part, out1, total;
};

GradLayout grad_layout(const nqs_model *m, int64_t n) {
  GradPlan g = grad_plan(m, n);
  const size_t es = (use_double(m) ? 8 : 4) * (m->is_complex ? 2 : 1);
  GradLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += (bytes + 255) / 256 * 256;
    return o;
  };
  const size_t elems = size_t(g.Jtiles) * 16 * size_t(g.Itiles) * 16;
  // FP32 direction tables are followed by their bf16 split (the JVP's B operand)
  L.Vt = take(vsplit_offset(m->N, m->M, es) +
              (use_double(m) ? 0 : vsplit_bytes(m->N, m->M, m->is_complex ? 2 : 1)));
  L.vb = take(size_t(m->M) * es);
  L.va = take(size_t(m->N) * 16);
  L.ypart = take(size_t(g.jchunks) * size_t(n) * 16);
  L.Tm = take(size_t(n) * m->M * es + 128 * es);  // slack: whole-tile reads past the last row
  L.masks = take(g.pair ? size_t(n) * 8 : 0);
  // spin quads of k_vjp_wide: [4 ceil(n / 16)][16 Itiles] uint2
  L.sq = take(g.wide ? size_t(4 * cdiv(n > 0 ? n : 1, 16)) * g.Itiles * 16 * 8 : 0);
  // sized for the largest split count any plan of this device uses, so that a later
  // change of the tuned S v shape never outgrows a workspace sized earlier
  const size_t splits_cap = size_t(g.splits) > size_t(2 * m->cu_count) ? size_t(g.splits)
                                                                        : size_t(2 * m->cu_count);
  L.part = take(splits_cap * elems * es);
  L.out1 = take(size_t(g.groups) * elems * 16);
  L.total = off;
  return L;
}

template <typename T, bool C>
hipError_t prep_t(const nqs_model *m, const void *v, void *scratch, bool split, hipStream_t st) {
  GradLayout L = grad_layout(m, 0);
  char *base = (char *)scratch;
  int64_t total = int64_t(m->N) * m->M + m->M + m->N;
  int blocks = int(cdiv(total, 256));
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL((k_prep_dir<T, C>), dim3(blocks), dim3(256), 0, st, m->N, m->M,
                     (const double *)v, (T *)(base + L.Vt), (T *)(base + L.vb),
                     (double *)(base + L.va), int(split));
  return hipGetLastError();
}

template <typename T, bool C>
hipError_t tanh_t(const nqs_model *m, const int8_t *sigma, int64_t n, void *scratch,
                  bool for_grad, hipStream_t st) {
  if (n == 0) return hipSuccess;
  GradPlan g = grad_plan(m, n);
  GradLayout L = grad_layout(m, n);
  char *base = (char *)scratch;
  hipLaunchKernelGGL((k_theta_tanh<T, C>), dim3(unsigned(g.jvp_blocks), g.jchunks), dim3(256),
                     0, st, m->N, m->M, n, sigma, (const T *)m->tab_ptrs[0],
                     (const T *)m->tab_ptrs[1],
                     for_grad && m->prec == NQS_BF16 ? (g.tbf ? 2 : 1) : 0,
                     int(m->prec == NQS_BF16), (T *)(base + L.Tm));
  if (g.pair) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_pack_spins, dim3(unsigned(cdiv(n, 256))), dim3(256), 0, st, m->N, n,
                       sigma, (uint64_t *)(base + L.masks));
  }
  if (g.wide && for_grad) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t groups = 4 * cdiv(n, 16);
    const int64_t b = cdiv(groups * g.Itiles * 16, 256);
    hipLaunchKernelGGL(k_sigma_quads, dim3(unsigned(b < 8192 ? b : 8192)), dim3(256), 0, st,
                       m->N, g.Itiles * 16, n, groups, sigma, (uint2 *)(base + L.sq));
  }
  return hipGetLastError();
}

template <typename T, bool C>
hipError_t jvp_t(const nqs_model *m, const int8_t *sigma, int64_t n, void *scratch, double *y,
                 double *ysum_part, const int *skip, hipStream_t st) {
  GradPlan g = grad_plan(m, n);
  GradLayout L = grad_layout(m, n);
  char *base = (char *)scratch;
  if constexpr (sizeof(T) == 4) {
    const int cw = jvp32_cw(g.jchunks);
    const dim3 grid(unsigned(cdiv(n > 0 ? n : 1, 256 / cw)), unsigned(cdiv(g.jchunks, cw)));
#define NQS_JVP32(TB)                                                                      \
  hipLaunchKernelGGL((k_jvp32<C, TB>), grid, dim3(256), 0, st, cw, g.jchunks, m->N, m->M, n,   \
                     sigma, (const T *)(base + L.Tm), (const T *)(base + L.Vt),                \
                     (const T *)(base + L.vb), (const double *)(base + L.va),                  \
                     (double *)(base + L.ypart), skip)
    if (g.tbf)
      NQS_JVP32(true);
    else
      NQS_JVP32(false);
#undef NQS_JVP32
  } else {
    hipLaunchKernelGGL((k_jvp<T, C>), dim3(unsigned(g.jvp_blocks), g.jchunks), dim3(256), 0, st,
                       m->N, m->M, n, sigma, (const T *)(base + L.Tm), (const T *)(base + L.Vt),
                       (const T *)(base + L.vb), (const double *)(base + L.va),
                       (double *)(base + L.ypart), skip);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_jvp_finish<C>), dim3(unsigned(cdiv(n, 256))), dim3(256), 0, st, n,
                     g.jchunks, (const double *)(base + L.ypart), y, ysum_part, skip);
  return hipGetLastError();
}

template <typename T, bool C, int JT, int NT>
hipError_t vjp_tile(const nqs_model *m, const int8_t *sigma, int64_t n, const double *u,
                    void *scratch, const int *skip, hipStream_t st, bool reduce) {
  GradPlan g = grad_plan(m, n);
  GradLayout L = grad_layout(m, n);
  char *base = (char *)scratch;
  const int gx = int(cdiv(g.Jtiles, JT)), gz = int(cdiv(g.Itiles, NT));
  const int64_t total = int64_t(gx) * g.splits * gz;
  const dim3 grid(unsigned(kXcds * cdiv(total, kXcds)));
#define NQS_VJPT(TB)                                                                          \
  hipLaunchKernelGGL((k_vjp<T, C, JT, NT, TB>), grid, dim3(256), 0, st, gx, gz, total, m->N,   \
                     m->M, n, sigma, (const T *)(base + L.Tm), u, g.per_split, g.Jtiles * 16,  \
                     g.Itiles * 16, (T *)(base + L.part), skip)
  bool done = false;
  if constexpr (C && sizeof(T) == 4) {
    if (g.tbf) {
      NQS_VJPT(true);
      done = true;
    }
  }
  if (!done) NQS_VJPT(false);
#undef NQS_VJPT
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !reduce) return e;
  const int64_t elems = int64_t(g.Jtiles) * 16 * g.Itiles * 16;
  hipLaunchKernelGGL((k_vjp_reduce1<T, C>), dim3(unsigned(cdiv(elems, 256)), g.groups),
                     dim3(256), 0, st, g.splits, g.groups, elems, (const T *)(base + L.part),
                     (double *)(base + L.out1), skip);
  return hipGetLastError();
}

template <bool C, int JT, int NT>
hipError_t vjp_wide(const nqs_model *m, int64_t n, const double *u, void *scratch,
                    const int *skip, hipStream_t st, bool reduce) {
  GradPlan g = grad_plan(m, n);
  GradLayout L = grad_layout(m, n);
  char *base = (char *)scratch;
  const int gx = int(cdiv(g.Jtiles, JT));
#define NQS_VJPW(TB)                                                                          \
  hipLaunchKernelGGL((k_vjp_wide<C, JT, NT, TB>), dim3(unsigned(int64_t(gx) * g.splits)),      \
                     dim3(256), 0, st, gx, g.Itiles, m->M, n, (const uint2 *)(base + L.sq),    \
                     g.Itiles * 16, (const float *)(base + L.Tm), u, g.per_split,              \
                     g.Jtiles * 16, (float *)(base + L.part), skip)
  if (g.tbf)
    NQS_VJPW(true);
  else
    NQS_VJPW(false);
#undef NQS_VJPW
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !reduce) return e;
  const int64_t elems = int64_t(g.Jtiles) * 16 * g.Itiles * 16;
  hipLaunchKernelGGL((k_vjp_reduce1<float, C>), dim3(unsigned(cdiv(elems, 256)), g.groups),
                     dim3(256), 0, st, g.splits, g.groups, elems, (const float *)(base + L.part),
                     (double *)(base + L.out1), skip);
  return hipGetLastError();
}

template <typename T, bool C>
hipError_t vjp_t(const nqs_model *m, const int8_t *sigma, int64_t n, const double *u,
                 void *scratch, const int *skip, hipStream_t st, bool reduce) {
  GradPlan g = grad_plan(m, n);
  if constexpr (sizeof(T) == 4) {
    if (g.wide) {
      if (g.JT == 2) return vjp_wide<C, 2, 8>(m, n, u, scratch, skip, st, reduce);
      return vjp_wide<C, 1, 17>(m, n, u, scratch, skip, st, reduce);
    }
  }
#define NQS_VJP_CASE(A, B) \
  if (g.JT == A && g.NT == B) return vjp_tile<T, C, A, B>(m, sigma, n, u, scratch, skip, st, reduce);
  NQS_VJP_CASE(1, 1)
  NQS_VJP_CASE(2, 1)
  NQS_VJP_CASE(4, 1)
  NQS_VJP_CASE(6, 1)
  NQS_VJP_CASE(8, 1)
  NQS_VJP_CASE(1, 2)
  NQS_VJP_CASE(2, 2)
  NQS_VJP_CASE(4, 2)
  NQS_VJP_CASE(6, 2)
  NQS_VJP_CASE(8, 2)
  NQS_VJP_CASE(1, 3)
  NQS_VJP_CASE(2, 3)
  NQS_VJP_CASE(4, 3)
  NQS_VJP_CASE(6, 3)
  NQS_VJP_CASE(1, 4)
  NQS_VJP_CASE(2, 4)
  NQS_VJP_CASE(4, 4)
#undef NQS_VJP_CASE
  return hipErrorInvalidValue;
}

template <int JT, int JV, int NT, int PAIRS, bool TB>
hipError_t svc_run(const nqs_model *m, const GradPlan &g, const GradLayout &L, int64_t n,
                   char *base, double *ysum_part, const int *skip, hipStream_t st) {
  const size_t lds = svc_dynamic_lds(m->N, m->M);
  // dynamic LDS beyond 64 KiB is opted into once per instantiation (up to the device limit
  // checked by grad_plan)
  static const hipError_t opt = hipFuncSetAttribute(
      reinterpret_cast<const void *>(&k_svc<float, JT, JV, NT, PAIRS, TB>),
      hipFuncAttributeMaxDynamicSharedMemorySize, m->max_lds - 24 * 1024);
  if (opt != hipSuccess) return opt;
  hipLaunchKernelGGL((k_svc<float, JT, JV, NT, PAIRS, TB>), dim3(unsigned(g.splits)),
                     dim3(128 * PAIRS), lds, st, m->N, m->M, n,
                     (const uint64_t *)(base + L.masks), (const float *)(base + L.Tm),
                     (const float *)(base + L.Vt), (const float *)(base + L.vb),
                     (const double *)(base + L.va), g.per_split, g.Jtiles * 16,
                     g.Itiles * 16, (float *)(base + L.part), ysum_part, skip);
  return hipGetLastError();
}

template <int JT, int JV, int NT, int PAIRS>
hipError_t svc_go(const nqs_model *m, int64_t n, void *scratch, double *ysum_part,
                  const int *skip, hipStream_t st, bool reduce) {
  GradPlan g = grad_plan(m, n);
  GradLayout L = grad_layout(m, n);
  char *base = (char *)scratch;
  hipError_t e = g.tbf ? svc_run<JT, JV, NT, PAIRS, true>(m, g, L, n, base, ysum_part, skip, st)
                       : svc_run<JT, JV, NT, PAIRS, false>(m, g, L, n, base, ysum_part, skip, st);
  if (e != hipSuccess || !reduce) return e;
  const int64_t elems = int64_t(g.Jtiles) * 16 * g.Itiles * 16;
  hipLaunchKernelGGL((k_vjp_reduce1<float, true>), dim3(unsigned(cdiv(elems, 256)), g.groups),
                     dim3(256), 0, st, g.splits, g.groups, elems,
                     (const float *)(base + L.part), (double *)(base + L.out1), skip);
  return hipGetLastError();
}

template <int JT, int NT>
hipError_t svc_pick(const nqs_model *m, int64_t n, void *scratch, double *ysum_part,
                    const int *skip, hipStream_t st, bool reduce) {
  const GradPlan g = grad_plan(m, n);
  const bool full = (m->M % 16) == 0;  // row M starts a tile of its own
  if constexpr (JT > 1) {
    if (full)
      return g.pairs == 4 ? svc_go<JT, JT - 1, NT, 4>(m, n, scratch, ysum_part, skip, st, reduce)
                          : svc_go<JT, JT - 1, NT, 2>(m, n, scratch, ysum_part, skip, st, reduce);
  }
  if (full) return hipErrorInvalidValue;
  return g.pairs == 4 ? svc_go<JT, JT, NT, 4>(m, n, scratch, ysum_part, skip, st, reduce)
                      : svc_go<JT, JT, NT, 2>(m, n, scratch, ysum_part, skip, st, reduce);
}

// plane-split S v for complex FP32 (grad_plan(...).pair): JT = Jtiles exactly
hipError_t svc_launch(const nqs_model *m, int64_t n, void *scratch, double *ysum_part,
                      const int *skip, hipStream_t st, bool reduce) {
  const GradPlan g = grad_plan(m, n);
#define NQS_SVC_CASE(A, B) \
  if (g.Jtiles == A && g.NT == B) return svc_pick<A, B>(m, n, scratch, ysum_part, skip, st, reduce);
  NQS_SVC_CASE(1, 1) NQS_SVC_CASE(1, 2) NQS_SVC_CASE(1, 3) NQS_SVC_CASE(1, 4)
  NQS_SVC_CASE(2, 1) NQS_SVC_CASE(2, 2) NQS_SVC_CASE(2, 3) NQS_SVC_CASE(2, 4)
  NQS_SVC_CASE(3, 1) NQS_SVC_CASE(3, 2) NQS_SVC_CASE(3, 3) NQS_SVC_CASE(3, 4)
  NQS_SVC_CASE(4, 1) NQS_SVC_CASE(4, 2) NQS_SVC_CASE(4, 3) NQS_SVC_CASE(4, 4)
  NQS_SVC_CASE(5, 1) NQS_SVC_CASE(5, 2) NQS_SVC_CASE(5, 3)
  NQS_SVC_CASE(6, 1) NQS_SVC_CASE(6, 2) NQS_SVC_CASE(6, 3)
#undef NQS_SVC_CASE
  return hipErrorInvalidValue;
}

template <typename T, bool C, int JT, int NT>
hipError_t sv_tile(const nqs_model *m, const int8_t *sigma, int64_t n, void *scratch,
                   double *ysum_part, const int *skip, hipStream_t st, bool reduce) {
  GradPlan g = grad_plan(m, n);
  GradLayout L = grad_layout(m, n);
  char *base = (char *)scratch;
  const int Kp = (m->N + 3) / 4 * 4;
  const size_t vbytes = (size_t(Kp) * JT * 16 * sizeof(T) * (C ? 2 : 1) + 15) / 16 * 16;
  const size_t tile_bytes = size_t(4) * 16 * NT * 16;
  hipLaunchKernelGGL((k_sv<T, C, JT, NT>), dim3(unsigned(g.splits)), dim3(256),
                     vbytes + tile_bytes, st, m->N, m->M, n, sigma, (const T *)(base + L.Tm),
                     (const T *)(base + L.Vt), (const T *)(base + L.vb),
                     (const double *)(base + L.va), g.per_split, g.Jtiles * 16, g.Itiles * 16,
                     (T *)(base + L.part), ysum_part, skip);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !reduce) return e;
  const int64_t elems = int64_t(g.Jtiles) * 16 * g.Itiles * 16;
  hipLaunchKernelGGL((k_vjp_reduce1<T, C>), dim3(unsigned(cdiv(elems, 256)), g.groups),
                     dim3(256), 0, st, g.splits, g.groups, elems, (const T *)(base + L.part),
                     (double *)(base + L.out1), skip);
  return hipGetLastError();
}

template <typename T, bool C>
hipError_t sv_t(const nqs_model *m, const int8_t *sigma, int64_t n, void *scratch,
                double *ysum_part, const int *skip, hipStream_t st, bool reduce) {
  GradPlan g = grad_plan(m, n);
  if constexpr (C && std::is_same<T, float>::value) {
    if (g.pair) return svc_launch(m, n, scratch, ysum_part, skip, st, reduce);
  }
#define NQS_SV_CASE(A, B) \
  if (g.JT == A && g.NT == B) return sv_tile<T, C, A, B>(m, sigma, n, scratch, ysum_part, skip, st, reduce);
  NQS_SV_CASE(1, 1)
  NQS_SV_CASE(2, 1)
  NQS_SV_CASE(4, 1)
  NQS_SV_CASE(6, 1)
  NQS_SV_CASE(8, 1)
  NQS_SV_CASE(1, 2)
  NQS_SV_CASE(2, 2)
  NQS_SV_CASE(4, 2)
  NQS_SV_CASE(6, 2)
  NQS_SV_CASE(8, 2)
  NQS_SV_CASE(1, 3)
  NQS_SV_CASE(2, 3)
  NQS_SV_CASE(4, 3)
  NQS_SV_CASE(6, 3)
  NQS_SV_CASE(1, 4)
  NQS_SV_CASE(2, 4)
  NQS_SV_CASE(4, 4)
#undef NQS_SV_CASE
  return hipErrorInvalidValue;
}

template <typename T, bool C>
hipError_t vjp_reduce_t(const nqs_model *m, int64_t n, void *scratch, double *out,
                        const int *skip, hipStream_t st) {
  GradPlan g = grad_plan(m, n);
  GradLayout L = grad_layout(m, n);
  char *base = (char *)scratch;
  int64_t P = int64_t(m->N) + m->M + int64_t(m->N) * m->M;
  int blocks = int(cdiv(P, 256));
  if (blocks > 8192) blocks = 8192;
  const int64_t elems = int64_t(g.Jtiles) * 16 * g.Itiles * 16;
  hipLaunchKernelGGL((k_vjp_reduce2<C>), dim3(blocks), dim3(256), 0, st, m->N, m->M, g.groups,
                     g.Itiles * 16, elems, (const double *)(base + L.out1), out, skip);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Batches of models (nqs_batch): one launch per kernel for every model. Each block reads
// its model's arguments from a job table and its block indices from a block map, then
// runs the single-model body. The VJP uses 4 x 2 output tiles per block and splits of
// 256 samples for every model.
// ---------------------------------------------------------------------------------
constexpr int kBJT = 4, kBNT = 2, kBSplit = 256;

template <typename T>
struct TanhJob {
  int N, M;
  int64_t n;
  const int8_t *sigma;
  const T *Wt, *bv;
  int quant, wbf;  // wbf: weights exact in bfloat16 (BF16 form)
  T *Tout;
};
template <typename T, bool C>
__global__ __launch_bounds__(256) void kb_theta_tanh(const TanhJob<T> *jobs, const int4 *map) {
  const int4 b = map[blockIdx.x];
  const TanhJob<T> J = jobs[b.x];
  k_theta_tanh_body<T, C>(b.y, b.z, 0, 0, J.N, J.M, J.n, J.sigma, J.Wt, J.bv, J.quant, J.wbf,
                          J.Tout);
}

template <typename T>
struct JvpJob {
  int N, M;
  int64_t n;
  const int8_t *sigma;
  const T *Tm, *Vt, *vb;
  const double *va;
  double *ypart, *y, *ysum;
  int jchunks, cw;  // cw: hidden chunks per block of the FP32 kernel
  const int *skip;
};
template <typename T, bool C>
__global__ __launch_bounds__(256, 2) void kb_jvp(const JvpJob<T> *jobs, const int4 *map) {
  const int4 b = map[blockIdx.x];
  const JvpJob<T> J = jobs[b.x];
  if constexpr (sizeof(T) == 4)
    k_jvp32_body<C>(b.y, b.z, J.cw, J.jchunks, J.N, J.M, J.n, J.sigma, J.Tm, J.Vt, J.vb, J.va,
                    J.ypart, J.skip);
  else
    k_jvp_body<T, C>(b.y, b.z, 0, 0, J.N, J.M, J.n, J.sigma, J.Tm, J.Vt, J.vb, J.va, J.ypart,
                     J.skip);
}
template <typename T, bool C>
__global__ __launch_bounds__(256) void kb_jvp_finish(const JvpJob<T> *jobs, const int4 *map) {
  const int4 b = map[blockIdx.x];
  const JvpJob<T> J = jobs[b.x];
  k_jvp_finish_body<C>(b.y, 0, 0, 0, J.n, J.jchunks, J.ypart, J.y, J.ysum, J.skip);
}

template <typename T>
struct VjpJob {
  int N, M;
  int64_t n;
  const int8_t *sigma;
  const T *Tm;
  const double *u;
  int rowsP, colsP, splits, pad0;  // explicit padding (zero): job tables are compared
  int64_t elems;                   // byte by byte before an upload
  T *part;
  double *out1;  // [rowsP][colsP] complex double
  double *out;   // packed like the parameters, or NULL (kept in out1)
  int pblocks, pad1;
  const int *skip;
};
template <typename T, bool C>
__global__ __launch_bounds__(256) void kb_vjp(const VjpJob<T> *jobs, const int4 *map) {
  const int4 b = map[blockIdx.x];
  const VjpJob<T> J = jobs[b.x];
  k_vjp_body<T, C, kBJT, kBNT>(b.y, b.z, b.w, 0, J.N, J.M, J.n, J.sigma, J.Tm, J.u, kBSplit,
                               J.rowsP, J.colsP, J.part, J.skip);
}
template <typename T, bool C>
__global__ __launch_bounds__(256) void kb_vjp_reduce1(const VjpJob<T> *jobs, const int4 *map) {
  const int4 b = map[blockIdx.x];
  const VjpJob<T> J = jobs[b.x];
  if (int64_t(b.y) * 256 + threadIdx.x >= J.elems) return;
  k_vjp_reduce1_body<T, C>(b.y, 0, 0, 0, J.splits, 1, J.elems, J.part, J.out1, J.skip);
}
template <typename T, bool C>
__global__ __launch_bounds__(256) void kb_vjp_reduce2(const VjpJob<T> *jobs, const int4 *map) {
  const int4 b = map[blockIdx.x];
  const VjpJob<T> J = jobs[b.x];
  k_vjp_reduce2_body<C>(b.y, 0, 0, J.pblocks, J.N, J.M, 1, J.colsP, J.elems, J.out1, J.out,
                        J.skip);
}

// job tables are compared byte by byte with the previous upload: no implicit padding
static_assert(std::has_unique_object_representations_v<TanhJob<float>> &&
                  std::has_unique_object_representations_v<JvpJob<float>> &&
                  std::has_unique_object_representations_v<VjpJob<float>> &&
                  std::has_unique_object_representations_v<JvpJob<double>> &&
                  std::has_unique_object_representations_v<VjpJob<double>>,
              "job structs must not hold padding bytes");

template <typename T>
hipError_t upload_launch_map(JobBuffer &jb, JobBuffer &mb, const std::vector<T> &jobs,
                             const std::vector<int4> &map, hipStream_t st) {
  hipError_t e = jb.upload(jobs.data(), jobs.size() * sizeof(T), st);
  if (e != hipSuccess) return e;
  if ((e = mb.upload(map.data(), map.size() * sizeof(int4), st)) != hipSuccess) return e;
  // never launch on a table that is not there
  if (!map.empty() && (!jb.d || !mb.d)) return hipErrorInvalidValue;
  return hipSuccess;
}

template <typename T, bool C>
hipError_t tanh_batch_t(nqs_batch *b, const std::vector<BatchGradItem> &items, int slot,
                        hipStream_t st) {
  std::vector<TanhJob<T>> jobs;
  std::vector<int4> map;
  for (size_t k = 0; k < items.size(); ++k) {
    const BatchGradItem &it = items[k];
    const nqs_model *m = it.m;
    TanhJob<T> J{m->N, m->M, it.n, it.sigma, (const T *)m->tab_ptrs[0], (const T *)m->tab_ptrs[1],
                 int(m->prec == NQS_BF16), int(m->prec == NQS_BF16), (T *)it.Tm};
    jobs.push_back(J);
    const int gx = int(cdiv(it.n, 64)), gy = int(cdiv((m->M + 15) / 16, Chunk<T, C>::JT));
    for (int y = 0; y < gy; ++y)
      for (int x = 0; x < gx; ++x) map.push_back(make_int4(int(k), x, y, 0));
  }
  hipError_t e = upload_launch_map(b->buf(slot), b->buf(slot + 1), jobs, map, st);
  if (e != hipSuccess || map.empty()) return e;
  hipLaunchKernelGGL((kb_theta_tanh<T, C>), dim3(unsigned(map.size())), dim3(256), 0, st,
                     (const TanhJob<T> *)b->buf(slot).d, (const int4 *)b->buf(slot + 1).d);
  return hipGetLastError();
}

template <typename T, bool C>
hipError_t jvp_batch_t(nqs_batch *b, const std::vector<BatchGradItem> &items, int slot,
                       hipStream_t st) {
  std::vector<JvpJob<T>> jobs;
  std::vector<int4> map, map2;
  for (size_t k = 0; k < items.size(); ++k) {
    const BatchGradItem &it = items[k];
    const nqs_model *m = it.m;
    const int jchunks = int(cdiv((m->M + 15) / 16, Chunk<T, C>::JT));
    const int cw = sizeof(T) == 4 ? jvp32_cw(jchunks) : 1;
    JvpJob<T> J{m->N, m->M, it.n, it.sigma, (const T *)it.Tm, (const T *)it.Vt, (const T *)it.vb,
                it.va, it.ypart, it.y, it.ysum, jchunks, cw, it.skip};
    jobs.push_back(J);
    const int gx = int(cdiv(it.n, sizeof(T) == 4 ? 256 / cw : 64));
    for (int y = 0; y < int(cdiv(jchunks, cw)); ++y)
      for (int x = 0; x < gx; ++x) map.push_back(make_int4(int(k), x, y, 0));
    for (int x = 0; x < int(cdiv(it.n, 256)); ++x) map2.push_back(make_int4(int(k), x, 0, 0));
  }
  hipError_t e = upload_launch_map(b->buf(slot), b->buf(slot + 1), jobs, map, st);
  if (e == hipSuccess) e = b->buf(slot + 2).upload(map2.data(), map2.size() * sizeof(int4), st);
  if (e != hipSuccess || map.empty()) return e;
  if (!b->buf(slot + 2).d) return hipErrorInvalidValue;
  hipLaunchKernelGGL((kb_jvp<T, C>), dim3(unsigned(map.size())), dim3(256), 0, st,
                     (const JvpJob<T> *)b->buf(slot).d, (const int4 *)b->buf(slot + 1).d);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL((kb_jvp_finish<T, C>), dim3(unsigned(map2.size())), dim3(256), 0, st,
                     (const JvpJob<T> *)b->buf(slot).d, (const int4 *)b->buf(slot + 2).d);
  return hipGetLastError();
}

template <typename T, bool C>
hipError_t vjp_batch_t(nqs_batch *b, const std::vector<BatchGradItem> &items, bool to_params,
                       int slot, hipStream_t st) {
  std::vector<VjpJob<T>> jobs;
  std::vector<int4> map, map1, map2;
  for (size_t k = 0; k < items.size(); ++k) {
    const BatchGradItem &it = items[k];
    const nqs_model *m = it.m;
    const int Jtiles = (m->M + 1 + 15) / 16, Itiles = (m->N + 1 + 15) / 16;
    const int splits = int(cdiv(it.n > 0 ? it.n : 1, kBSplit));
    const int64_t elems = int64_t(Jtiles) * 16 * Itiles * 16;
    const int64_t P = int64_t(m->N) + m->M + int64_t(m->N) * m->M;
    const int pblocks = int(cdiv(P, 256) < 4096 ? cdiv(P, 256) : 4096);
    VjpJob<T> J{m->N,  m->M,    it.n,         it.sigma,  (const T *)it.Tm, it.u,
                Jtiles * 16, Itiles * 16, splits, 0, elems, (T *)it.part, it.out1,
                to_params ? it.out : nullptr, pblocks, 0, it.skip};
    jobs.push_back(J);
    for (int z = 0; z < int(cdiv(Itiles, kBNT)); ++z)
      for (int y = 0; y < splits; ++y)
        for (int x = 0; x < int(cdiv(Jtiles, kBJT)); ++x)
          map.push_back(make_int4(int(k), x, y, z));
    for (int x = 0; x < int(cdiv(elems, 256)); ++x) map1.push_back(make_int4(int(k), x, 0, 0));
    for (int x = 0; x < pblocks; ++x) map2.push_back(make_int4(int(k), x, 0, 0));
  }
  hipError_t e = upload_launch_map(b->buf(slot), b->buf(slot + 1), jobs, map, st);
  if (e == hipSuccess) e = b->buf(slot + 2).upload(map1.data(), map1.size() * sizeof(int4), st);
  if (e == hipSuccess && to_params)
    e = b->buf(slot + 3).upload(map2.data(), map2.size() * sizeof(int4), st);
  if (e != hipSuccess || map.empty()) return e;
  if (!b->buf(slot + 2).d || (to_params && !b->buf(slot + 3).d)) return hipErrorInvalidValue;
  const VjpJob<T> *dj = (const VjpJob<T> *)b->buf(slot).d;
  hipLaunchKernelGGL((kb_vjp<T, C>), dim3(unsigned(map.size())), dim3(256), 0, st, dj,
                     (const int4 *)b->buf(slot + 1).d);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL((kb_vjp_reduce1<T, C>), dim3(unsigned(map1.size())), dim3(256), 0, st, dj,
                     (const int4 *)b->buf(slot + 2).d);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (to_params) {
    hipLaunchKernelGGL((kb_vjp_reduce2<T, C>), dim3(unsigned(map2.size())), dim3(256), 0, st,
                       dj, (const int4 *)b->buf(slot + 3).d);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace

GradPlan grad_plan(const nqs_model *m, int64_t n) {
  GradPlan g;
  g.Jtiles = (m->M + 1 + 15) / 16;   // hidden rows 0..M (row M carries the visible bias)
  g.Itiles = (m->N + 1 + 15) / 16;   // site columns 0..N (column N carries the hidden bias)
  g.NT = g.Itiles < 4 ? g.Itiles : 4;
  // accumulator tiles per wavefront: <= 24, <= 16 with 4 site tiles (the instantiated
  // (JT, NT) pairs of k_vjp / k_sv)
  const int jt_budget = (g.NT == 4 ? 16 : 24) / g.NT;
  static const int jts[5] = {8, 6, 4, 2, 1};
  g.JT = 1;
  for (int q = 0; q < 5; ++q)
    if (jts[q] <= jt_budget && (jts[q] <= g.Jtiles || q == 4)) {
      g.JT = jts[q];
      break;
    }
  if (g.NT == 3 && g.JT == 8) g.JT = 6;
  const int64_t tile_blocks = cdiv(g.Jtiles, g.JT) * cdiv(g.Itiles, g.NT);
  const int64_t steps = n > 0 ? cdiv(n, 16) : 1;   // 16 samples = one step of all 4 waves
  int64_t splits = 2 * int64_t(m->cu_count) / tile_blocks;
  if (splits < 1) splits = 1;
  if (splits > steps) splits = steps;
  g.per_split = rup(cdiv(n > 0 ? n : 1, splits), 16);
  g.splits = int(cdiv(n > 0 ? n : 1, g.per_split));
  {
    const size_t es = (use_double(m) ? 8 : 4) * (m->is_complex ? 2 : 1);
    const size_t vbytes = size_t((m->N + 3) / 4 * 4) * g.JT * 16 * es;
    g.fused = tile_blocks == 1 && vbytes <= 48 * 1024;
  }
  // complex FP32 with N <= 63: the plane-split fused product (k_svc) with the smallest
  // hidden-tile count covering rows 0..M, at most 6 x 3 accumulator tiles per wavefront
  g.pair = false;
  if (m->is_complex && !use_double(m) && m->N <= 63 && g.Jtiles <= 6 &&
      g.Jtiles * g.NT <= 18) {
    // dynamic LDS of the 4-pair shape plus the kernel's static arrays (<= 24 KiB)
    const size_t lds = svc_dynamic_lds(m->N, m->M) + 24 * 1024;
    if (lds <= size_t(m->max_lds)) {
      g.pair = true;
      g.fused = true;
      // the separate k_vjp (O^dagger 1, force) takes the smallest tile count covering
      // every hidden row in one block
      static const int pj[4] = {1, 2, 4, 6};
      for (int q = 0; q < 4; ++q)
        if (pj[q] >= g.Jtiles) {
          g.JT = pj[q];
          break;
        }
    }
  }
  g.pairs = g.pair ? (m->sv_pairs == 4 ? 4 : 2) : 0;
  // FP32 / BF16 with 5 to 17 site tiles: every site tile in one block (k_vjp_wide), 2 (up
  // to 8 tiles) or 1 hidden tiles per block, two blocks per compute unit
  g.wide = false;
  if (!g.fused && !use_double(m) && g.Itiles >= 5 && g.Itiles <= 17) {
    g.wide = true;
    g.JT = g.Itiles <= 8 ? 2 : 1;
    g.NT = g.Itiles;
    const int64_t tb = cdiv(g.Jtiles, g.JT);
    int64_t sp = 2 * int64_t(m->cu_count) / tb;
    if (sp < 1) sp = 1;
    if (sp > steps) sp = steps;
    g.per_split = rup(cdiv(n > 0 ? n : 1, sp), 16);
    g.splits = int(cdiv(n > 0 ? n : 1, g.per_split));
  }
  // the BF16 form keeps its (bfloat16) T rows for the Jacobian products in 2 bytes per
  // value where every kernel that reads them can: k_jvp32 with k_vjp_wide, or with k_svc
  // and k_vjp (complex)
  g.tbf = m->prec == NQS_BF16 && (g.wide || g.pair);
  if (g.fused) {
    // fused S v: two blocks of 4 wavefronts per compute unit (one of 8 with 4 pairs),
    // splits of whole 16-sample groups
    int64_t sp = g.pairs == 4 ? int64_t(m->cu_count) : 2 * int64_t(m->cu_count);
    const int64_t groups16 = n > 0 ? cdiv(n, 16) : 1;
    if (sp > groups16) sp = groups16;
    g.per_split = rup(cdiv(n > 0 ? n : 1, sp), 16);
    g.splits = int(cdiv(n > 0 ? n : 1, g.per_split));
  }
  g.groups = g.splits < 16 ? g.splits : 16;
  g.jchunks = int(cdiv((m->M + 15) / 16, (use_double(m) || m->is_complex) ? 4 : 8));
  g.jvp_blocks = cdiv(n > 0 ? n : 1, 64);
  return g;
}

size_t grad_scratch_bytes(const nqs_model *m, int64_t n) { return grad_layout(m, n).total; }

#define NQS_DISPATCH(FN, ...)                                                              \
  (use_double(m) ? (m->is_complex ? FN<double, true>(__VA_ARGS__)                          \
                                  : FN<double, false>(__VA_ARGS__))                        \
                 : (m->is_complex ? FN<float, true>(__VA_ARGS__)                           \
                                  : FN<float, false>(__VA_ARGS__)))

hipError_t launch_prep_dir(const nqs_model *m, const void *v, void *scratch, bool split,
                           hipStream_t st) {
  return NQS_DISPATCH(prep_t, m, v, scratch, split, st);
}

hipError_t launch_theta_tanh(const nqs_model *m, const int8_t *sigma, int64_t n, void *scratch,
                             bool for_grad, hipStream_t st) {
  return NQS_DISPATCH(tanh_t, m, sigma, n, scratch, for_grad, st);
}

hipError_t launch_jvp(const nqs_model *m, const int8_t *sigma, int64_t n, void *scratch,
                      double *y, double *ysum_part, const int *skip, hipStream_t st) {
  return NQS_DISPATCH(jvp_t, m, sigma, n, scratch, y, ysum_part, skip, st);
}

hipError_t launch_vjp_partials(const nqs_model *m, const int8_t *sigma, int64_t n,
                               const double *u, void *scratch, const int *skip,
                               hipStream_t st, bool reduce) {
  return NQS_DISPATCH(vjp_t, m, sigma, n, u, scratch, skip, st, reduce);
}

hipError_t launch_sv(const nqs_model *m, const int8_t *sigma, int64_t n, void *scratch,
                     double *ysum_part, const int *skip, hipStream_t st, bool reduce) {
  return NQS_DISPATCH(sv_t, m, sigma, n, scratch, ysum_part, skip, st, reduce);
}

GradBuffers grad_buffers(const nqs_model *m, int64_t n, void *scratch) {
  GradLayout L = grad_layout(m, n);
  char *base = (char *)scratch;
  GradBuffers b;
  b.Tm = base + L.Tm;
  b.Vt = base + L.Vt;
  b.vb = base + L.vb;
  b.va = (double *)(base + L.va);
  b.out1 = (double *)(base + L.out1);
  b.part = base + L.part;
  return b;
}

hipError_t launch_vjp_reduce(const nqs_model *m, int64_t n, void *scratch, double *out,
                             const int *skip, hipStream_t st) {
  return NQS_DISPATCH(vjp_reduce_t, m, n, scratch, out, skip, st);
}

BatchGradSizes batch_grad_sizes(const nqs_model *m, int64_t n) {
  BatchGradSizes z;
  const size_t es = (use_double(m) ? 8 : 4) * (m->is_complex ? 2 : 1);
  const int Jtiles = (m->M + 1 + 15) / 16, Itiles = (m->N + 1 + 15) / 16;
  const int64_t splits = cdiv(n > 0 ? n : 1, kBSplit);
  z.Tm = size_t(n) * m->M * es + 128 * es;
  z.Vt = vsplit_offset(m->N, m->M, es) +
         (use_double(m) ? 0 : vsplit_bytes(m->N, m->M, m->is_complex ? 2 : 1));
  z.vb = size_t(m->M) * es;
  z.va = size_t(m->N) * 16;
  z.ypart = size_t(cdiv((m->M + 15) / 16, (use_double(m) || m->is_complex) ? 4 : 8)) *
            size_t(n) * 16;
  z.part = size_t(splits) * Jtiles * 16 * Itiles * 16 * es;
  z.out1 = size_t(Jtiles) * 16 * Itiles * 16 * 16;
  z.colsP = Itiles * 16;
  z.elems = int64_t(Jtiles) * 16 * Itiles * 16;
  return z;
}

hipError_t launch_theta_tanh_batch(nqs_batch *b, const std::vector<BatchGradItem> &items,
                                   int slot, hipStream_t st) {
  if (items.empty()) return hipSuccess;
  const nqs_model *m = items[0].m;
  return NQS_DISPATCH(tanh_batch_t, b, items, slot, st);
}

hipError_t launch_jvp_batch(nqs_batch *b, const std::vector<BatchGradItem> &items, int slot,
                            hipStream_t st) {
  if (items.empty()) return hipSuccess;
  const nqs_model *m = items[0].m;
  return NQS_DISPATCH(jvp_batch_t, b, items, slot, st);
}

hipError_t launch_vjp_batch(nqs_batch *b, const std::vector<BatchGradItem> &items,
                            bool to_params, int slot, hipStream_t st) {
  if (items.empty()) return hipSuccess;
  const nqs_model *m = items[0].m;
  return NQS_DISPATCH(vjp_batch_t, b, items, to_params, slot, st);
}
