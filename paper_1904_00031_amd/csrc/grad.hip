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
// FP64 MFMA (A: lane l holds A[l%16][l/16]; B: B[l/16][l%16]; D: lane l register r
// holds D[4(l/16)+r][l%16]).
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
};
template <>
struct MF<double> {
  typedef doublex4 acc;
  static __device__ __forceinline__ acc mma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t rup(int64_t a, int64_t b) { return cdiv(a, b) * b; }

// ---------------------------------------------------------------------------------
// Direction v (double, packed like the parameters) -> compute-precision tables.
// ---------------------------------------------------------------------------------
template <typename T, bool C>
__global__ void k_prep_dir(int N, int M, const double *__restrict__ v, T *Vt, T *vb,
                           double *va) {
  const int64_t total = int64_t(N) * M + M + N;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    if (e < int64_t(N) * M) {
      int j = int(e / N), i = int(e % N);  // read v_W row-major (j, i)
      vstore<T, C>(Vt, int64_t(i) * M + j, vcast<double, C, T>(vload<double, C>(v, N + M + e)));
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
// JVP. Grid (ceil(n/64), hidden chunks). Writes ypart[chunk][s] (complex double).
// ---------------------------------------------------------------------------------
template <typename T, bool C>
__global__ __launch_bounds__(256) void k_jvp(int N, int M, int64_t n,
                                              const int8_t *__restrict__ sigma,
                                              const T *__restrict__ Wt, const T *__restrict__ bv,
                                              const T *__restrict__ Vt, const T *__restrict__ vb,
                                              const double *__restrict__ va, int JT,
                                              double *ypart, const int *skip) {
  if (skip && *skip) return;
  typedef typename MF<T>::acc Acc;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int lo = lane & 15, hi = lane >> 4;
  const int64_t s0 = int64_t(blockIdx.x) * 64 + wid * 16;
  const int jc = blockIdx.y;
  const int ntiles = (M + 15) / 16;
  const int jt0 = jc * JT;
  const int jt1 = jt0 + JT < ntiles ? jt0 + JT : ntiles;
  const int64_t rowA = s0 + lo;
  const bool rowA_ok = rowA < n;
  const int8_t *srow = sigma + (rowA_ok ? rowA : 0) * N;
  V<T, C> yp[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) yp[r] = vmake<T, C>(T(0), T(0));
  for (int jt = jt0; jt < jt1; ++jt) {
    const int j = jt * 16 + lo;
    const bool jok = j < M;
    Acc tr = {0, 0, 0, 0}, ti = {0, 0, 0, 0}, xr = {0, 0, 0, 0}, xi = {0, 0, 0, 0};
    for (int k0 = 0; k0 < N; k0 += 4) {
      const int k = k0 + hi;
      const bool kok = k < N;
      const T a = (rowA_ok && kok) ? T(srow[k]) : T(0);
      V<T, C> w = vmake<T, C>(T(0), T(0)), v = vmake<T, C>(T(0), T(0));
      if (kok && jok) {
        w = vload<T, C>(Wt, int64_t(k) * M + j);
        v = vload<T, C>(Vt, int64_t(k) * M + j);
      }
      tr = MF<T>::mma(a, w.re, tr);
      xr = MF<T>::mma(a, v.re, xr);
      if constexpr (C) {
        ti = MF<T>::mma(a, w.im, ti);
        xi = MF<T>::mma(a, v.im, xi);
      }
    }
    if (jok) {
      const V<T, C> bb = vload<T, C>(bv, j), vbj = vload<T, C>(vb, j);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        V<T, C> th = vmake<T, C>(tr[r] + bb.re, C ? ti[r] + bb.im : T(0));
        V<T, C> x = vmake<T, C>(xr[r] + vbj.re, C ? xi[r] + vbj.im : T(0));
        yp[r] = vadd(yp[r], vmul(vtanh<T, C>(th), x));
      }
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
  if (lo == 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = s0 + 4 * hi + r;
      if (row >= n) continue;
      double yr = double(yp[r].re), yi = C ? double(yp[r].im) : 0.0;
      if (jc == 0) {
        const int8_t *sr = sigma + row * N;
        for (int i = 0; i < N; ++i) {
          yr += va[2 * i] * double(sr[i]);
          yi += va[2 * i + 1] * double(sr[i]);
        }
      }
      ypart[2 * (int64_t(jc) * n + row)] = yr;
      ypart[2 * (int64_t(jc) * n + row) + 1] = yi;
    }
  }
}

// y[s] = sum over chunks; per-block partial sums of y (complex double) for centering
template <bool C>
__global__ __launch_bounds__(256) void k_jvp_finish(int64_t n, int jchunks,
                                                     const double *__restrict__ ypart,
                                                     double *y, double *ysum_part,
                                                     const int *skip) {
  if (skip && *skip) return;
  __shared__ double sr[256], si[256];
  const int64_t s = int64_t(blockIdx.x) * 256 + threadIdx.x;
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
      ysum_part[2 * blockIdx.x] = sr[0];
      ysum_part[2 * blockIdx.x + 1] = si[0];
    }
  }
}

// ---------------------------------------------------------------------------------
// VJP partials. Grid (Mt hidden tiles incl. the extra row M that carries g_a, sample
// splits, site chunks). Each wavefront walks 16-sample groups: theta tile by MFMA,
// Z = conj(tanh theta) u in registers, a 16x16 transpose through LDS, then Z^T S by
// MFMA into NT site tiles. The four wavefronts of a block are summed through LDS.
// partW [split][Mt*16][Ncols], partB [split][Mt*16] (compute precision).
// ---------------------------------------------------------------------------------
template <typename T, bool C, int NT>
__global__ __launch_bounds__(256) void k_vjp(int N, int M, int64_t n,
                                              const int8_t *__restrict__ sigma,
                                              const T *__restrict__ Wt, const T *__restrict__ bv,
                                              const double *__restrict__ u, int64_t per_split,
                                              int Ncols, T *partW, T *partB, const int *skip) {
  if (skip && *skip) return;
  typedef typename MF<T>::acc Acc;
  __shared__ T zre[4][256];
  __shared__ T zim[4][C ? 256 : 1];
  __shared__ T red[4][4][64][C ? 2 : 1];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int lo = lane & 15, hi = lane >> 4;
  const int jt = blockIdx.x, split = blockIdx.y, zc = blockIdx.z;
  const int Mrows = gridDim.x * 16;
  const int j = jt * 16 + lo;
  const bool jok = j < M;
  const int i_base = zc * NT * 16;
  const int64_t sbeg = int64_t(split) * per_split;
  const int64_t send = sbeg + per_split < n ? sbeg + per_split : n;
  Acc ar[NT], ai[NT];
#pragma unroll
  for (int it = 0; it < NT; ++it) {
    ar[it] = Acc{0, 0, 0, 0};
    ai[it] = Acc{0, 0, 0, 0};
  }
  V<T, C> bsum = vmake<T, C>(T(0), T(0));
  const V<T, C> bb = jok ? vload<T, C>(bv, j) : vmake<T, C>(T(0), T(0));
  for (int64_t g = sbeg + wid * 16; g < send; g += 64) {
    const int64_t rowA = g + lo;
    const bool rowA_ok = rowA < send;
    const int8_t *srow = sigma + (rowA_ok ? rowA : 0) * N;
    Acc tr = {0, 0, 0, 0}, ti = {0, 0, 0, 0};
    for (int k0 = 0; k0 < N; k0 += 4) {
      const int k = k0 + hi;
      const bool kok = k < N;
      const T a = (rowA_ok && kok) ? T(srow[k]) : T(0);
      V<T, C> w = vmake<T, C>(T(0), T(0));
      if (kok && jok) w = vload<T, C>(Wt, int64_t(k) * M + j);
      tr = MF<T>::mma(a, w.re, tr);
      if constexpr (C) ti = MF<T>::mma(a, w.im, ti);
    }
    V<T, C> z[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = g + 4 * hi + r;
      z[r] = vmake<T, C>(T(0), T(0));
      if (row < send) {
        V<T, C> uu = vmake<T, C>(T(u[C ? 2 * row : row]), C ? T(u[2 * row + 1]) : T(0));
        if (jok) {
          V<T, C> th = vmake<T, C>(tr[r] + bb.re, C ? ti[r] + bb.im : T(0));
          z[r] = vmul(vconj(vtanh<T, C>(th)), uu);
          bsum = vadd(bsum, z[r]);
        } else if (j == M) {
          z[r] = uu;
        }
      }
    }
    wave_sync();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      zre[wid][(4 * hi + r) * 16 + lo] = z[r].re;
      if constexpr (C) zim[wid][(4 * hi + r) * 16 + lo] = z[r].im;
    }
    wave_sync();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const T a2r = zre[wid][(4 * q + hi) * 16 + lo];
      T a2i = T(0);
      if constexpr (C) a2i = zim[wid][(4 * q + hi) * 16 + lo];
      const int64_t srw = g + 4 * q + hi;
      const bool sok = srw < send;
      const int8_t *sp = sigma + (sok ? srw : 0) * N;
#pragma unroll
      for (int it = 0; it < NT; ++it) {
        const int i = i_base + it * 16 + lo;
        const T b2 = (sok && i < N) ? T(sp[i]) : T(0);
        ar[it] = MF<T>::mma(a2r, b2, ar[it]);
        if constexpr (C) ai[it] = MF<T>::mma(a2i, b2, ai[it]);
      }
    }
  }
  // column sums of Z for g_b: reduce over the four lane groups
  bsum.re += __shfl_xor(bsum.re, 16, 64);
  bsum.re += __shfl_xor(bsum.re, 32, 64);
  if constexpr (C) {
    bsum.im += __shfl_xor(bsum.im, 16, 64);
    bsum.im += __shfl_xor(bsum.im, 32, 64);
  }
  // sum the four wavefronts of the block, one site tile at a time
  const int tid = threadIdx.x;
  for (int it = 0; it < NT; ++it) {
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      red[wid][r][lane][0] = ar[it][r];
      if constexpr (C) red[wid][r][lane][C ? 1 : 0] = ai[it][r];
    }
    __syncthreads();
    // 256 threads cover 4 registers x 64 lanes
    const int r = tid >> 6, l = tid & 63;
    T sr = red[0][r][l][0] + red[1][r][l][0] + red[2][r][l][0] + red[3][r][l][0];
    T si = T(0);
    if constexpr (C)
      si = red[0][r][l][C ? 1 : 0] + red[1][r][l][C ? 1 : 0] + red[2][r][l][C ? 1 : 0] +
           red[3][r][l][C ? 1 : 0];
    const int jrow = jt * 16 + 4 * (l >> 4) + r;
    const int icol = i_base + it * 16 + (l & 15);
    const int64_t o = (int64_t(split) * Mrows + jrow) * Ncols + icol;
    if constexpr (C) {
      partW[2 * o] = sr;
      partW[2 * o + 1] = si;
    } else {
      partW[o] = sr;
    }
  }
  if (zc == 0) {
    __syncthreads();
    if (hi == 0) {
      red[wid][0][lo][0] = bsum.re;
      if constexpr (C) red[wid][0][lo][C ? 1 : 0] = bsum.im;
    }
    __syncthreads();
    if (tid < 16) {
      T sr = red[0][0][tid][0] + red[1][0][tid][0] + red[2][0][tid][0] + red[3][0][tid][0];
      const int64_t o = int64_t(split) * Mrows + jt * 16 + tid;
      if constexpr (C) {
        T si = red[0][0][tid][C ? 1 : 0] + red[1][0][tid][C ? 1 : 0] +
               red[2][0][tid][C ? 1 : 0] + red[3][0][tid][C ? 1 : 0];
        partB[2 * o] = sr;
        partB[2 * o + 1] = si;
      } else {
        partB[o] = sr;
      }
    }
  }
}

// out[k] (double, packed like the parameters) = sum over splits of the partials
template <typename T, bool C>
__global__ void k_vjp_reduce(int N, int M, int splits, int Mrows, int Ncols,
                             const T *__restrict__ partW, const T *__restrict__ partB,
                             double *out, const int *skip) {
  if (skip && *skip) return;
  const int64_t P = int64_t(N) + M + int64_t(N) * M;
  for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < P;
       k += int64_t(gridDim.x) * blockDim.x) {
    double sr = 0.0, si = 0.0;
    if (k < N + M && k >= N) {
      const int j = int(k - N);
      for (int p = 0; p < splits; ++p) {
        V<T, C> x = vload<T, C>(partB, int64_t(p) * Mrows + j);
        sr += double(x.re);
        si += double(x.im);
      }
    } else {
      int j, i;
      if (k < N) {
        j = M;
        i = int(k);
      } else {
        const int64_t q = k - N - M;
        j = int(q / N);
        i = int(q % N);
      }
      for (int p = 0; p < splits; ++p) {
        V<T, C> x = vload<T, C>(partW, (int64_t(p) * Mrows + j) * Ncols + i);
        sr += double(x.re);
        si += double(x.im);
      }
    }
    if (C) {
      out[2 * k] = sr;
      out[2 * k + 1] = si;
    } else {
      out[k] = sr;
    }
  }
}

// ---------------------------------------------------------------------------------
// scratch layout (byte offsets), all regions 256-byte aligned
// ---------------------------------------------------------------------------------
struct GradLayout {
  size_t Vt, vb, va, ypart, partW, partB, total;
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
  L.Vt = take(size_t(m->N) * m->M * es);
  L.vb = take(size_t(m->M) * es);
  L.va = take(size_t(m->N) * 16);
  L.ypart = take(size_t(g.jchunks) * size_t(n) * 16);
  L.partW = take(size_t(g.splits) * g.Mt * 16 * size_t(g.Nz * g.Nt * 16) * es);
  L.partB = take(size_t(g.splits) * g.Mt * 16 * es);
  L.total = off;
  return L;
}

template <typename T, bool C>
hipError_t prep_t(const nqs_model *m, const void *v, void *scratch, hipStream_t st) {
  GradLayout L = grad_layout(m, 0);
  char *base = (char *)scratch;
  int64_t total = int64_t(m->N) * m->M + m->M + m->N;
  int blocks = int(cdiv(total, 256));
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL((k_prep_dir<T, C>), dim3(blocks), dim3(256), 0, st, m->N, m->M,
                     (const double *)v, (T *)(base + L.Vt), (T *)(base + L.vb),
                     (double *)(base + L.va));
  return hipGetLastError();
}

template <typename T, bool C>
hipError_t jvp_t(const nqs_model *m, const int8_t *sigma, int64_t n, void *scratch, double *y,
                 double *ysum_part, const int *skip, hipStream_t st) {
  GradPlan g = grad_plan(m, n);
  GradLayout L = grad_layout(m, n);
  char *base = (char *)scratch;
  const T *Wt = (const T *)m->tab_ptrs[0];
  const T *bv = (const T *)m->tab_ptrs[1];
  hipLaunchKernelGGL((k_jvp<T, C>), dim3(unsigned(g.jvp_blocks), g.jchunks), dim3(256), 0, st,
                     m->N, m->M, n, sigma, Wt, bv, (const T *)(base + L.Vt),
                     (const T *)(base + L.vb), (const double *)(base + L.va), 16,
                     (double *)(base + L.ypart), skip);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_jvp_finish<C>), dim3(unsigned(cdiv(n, 256))), dim3(256), 0, st, n,
                     g.jchunks, (const double *)(base + L.ypart), y, ysum_part, skip);
  return hipGetLastError();
}

template <typename T, bool C, int NT>
hipError_t vjp_nt(const nqs_model *m, const int8_t *sigma, int64_t n, const double *u,
                  void *scratch, const int *skip, hipStream_t st) {
  GradPlan g = grad_plan(m, n);
  GradLayout L = grad_layout(m, n);
  char *base = (char *)scratch;
  const T *Wt = (const T *)m->tab_ptrs[0];
  const T *bv = (const T *)m->tab_ptrs[1];
  hipLaunchKernelGGL((k_vjp<T, C, NT>), dim3(g.Mt, g.splits, g.Nz), dim3(256), 0, st, m->N,
                     m->M, n, sigma, Wt, bv, u, g.per_split, g.Nz * g.Nt * 16,
                     (T *)(base + L.partW), (T *)(base + L.partB), skip);
  return hipGetLastError();
}

template <typename T, bool C>
hipError_t vjp_t(const nqs_model *m, const int8_t *sigma, int64_t n, const double *u,
                 void *scratch, const int *skip, hipStream_t st) {
  switch (grad_plan(m, n).Nt) {
    case 1: return vjp_nt<T, C, 1>(m, sigma, n, u, scratch, skip, st);
    case 2: return vjp_nt<T, C, 2>(m, sigma, n, u, scratch, skip, st);
    case 4: return vjp_nt<T, C, 4>(m, sigma, n, u, scratch, skip, st);
    case 8: return vjp_nt<T, C, 8>(m, sigma, n, u, scratch, skip, st);
    default: return vjp_nt<T, C, 16>(m, sigma, n, u, scratch, skip, st);
  }
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
  hipLaunchKernelGGL((k_vjp_reduce<T, C>), dim3(blocks), dim3(256), 0, st, m->N, m->M,
                     g.splits, g.Mt * 16, g.Nz * g.Nt * 16, (const T *)(base + L.partW),
                     (const T *)(base + L.partB), out, skip);
  return hipGetLastError();
}

}  // namespace

GradPlan grad_plan(const nqs_model *m, int64_t n) {
  GradPlan g;
  g.Mt = (m->M + 1 + 15) / 16;
  const int tilesN = (m->N + 15) / 16;
  int nt = 1;
  while (nt < tilesN && nt < 16) nt <<= 1;
  g.Nt = nt;
  g.Nz = int(cdiv(tilesN, nt));
  const int64_t groups = n > 0 ? cdiv(n, 64) : 1;
  int64_t splits = 2048 / (int64_t(g.Mt) * g.Nz);
  if (splits < 1) splits = 1;
  if (splits > groups) splits = groups;
  g.per_split = rup(cdiv(n > 0 ? n : 1, splits), 64);
  g.splits = int(cdiv(n > 0 ? n : 1, g.per_split));
  g.jchunks = int(cdiv((m->M + 15) / 16, 16));
  g.jvp_blocks = cdiv(n > 0 ? n : 1, 64);
  return g;
}

size_t grad_scratch_bytes(const nqs_model *m, int64_t n) { return grad_layout(m, n).total; }

#define NQS_DISPATCH(FN, ...)                                                              \
  (use_double(m) ? (m->is_complex ? FN<double, true>(__VA_ARGS__)                          \
                                  : FN<double, false>(__VA_ARGS__))                        \
                 : (m->is_complex ? FN<float, true>(__VA_ARGS__)                           \
                                  : FN<float, false>(__VA_ARGS__)))

hipError_t launch_prep_dir(const nqs_model *m, const void *v, void *scratch, hipStream_t st) {
  return NQS_DISPATCH(prep_t, m, v, scratch, st);
}

hipError_t launch_jvp(const nqs_model *m, const int8_t *sigma, int64_t n, void *scratch,
                      double *y, double *ysum_part, const int *skip, hipStream_t st) {
  return NQS_DISPATCH(jvp_t, m, sigma, n, scratch, y, ysum_part, skip, st);
}

hipError_t launch_vjp_partials(const nqs_model *m, const int8_t *sigma, int64_t n,
                               const double *u, void *scratch, const int *skip,
                               hipStream_t st) {
  return NQS_DISPATCH(vjp_t, m, sigma, n, u, scratch, skip, st);
}

hipError_t launch_vjp_reduce(const nqs_model *m, int64_t n, void *scratch, double *out,
                             const int *skip, hipStream_t st) {
  return NQS_DISPATCH(vjp_reduce_t, m, n, scratch, out, skip, st);
}

const double *scratch_vjp_partials(const nqs_model *m, int64_t n, void *scratch) {
  return (const double *)((char *)scratch + grad_layout(m, n).partW);
}
