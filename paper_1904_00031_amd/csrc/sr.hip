// Stochastic reconfiguration (Sec. 2.2.5: SR with an iterative solver; parameter step of
// Eq. 2). Given samples s and their local energies E_s:
//   E = <E_loc>, F = O^dagger (E - E) / n, (S + lambda I) x = F,
//   S v = O^dagger (O v - mean(O v)) / n = (O^dagger y - mean(y) O^dagger 1) / n,
// solved by conjugate gradients with every vector and scalar in double; the matrix-vector
// products run through the JVP/VJP kernels in the model's compute precision.
// All reductions are two-level (per-block partials, then every consumer block sums the
// partials in a fixed order), so results are bitwise reproducible run to run.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "internal.hpp"

namespace {

struct CGState {
  double E[2];
  double var;
  double err;  // error bar of Re E from the chain means
  double bnorm;
  double rr[2];  // r^dagger r, double-buffered by iteration parity
  double alpha;
  double fnorm;
  int iters;
  int done;
  int converged;
  int nonfinite;
};

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// block-level sum of per-thread values, identical in every thread (fixed order): DPP
// sums inside each wavefront, then the wavefront sums in index order. lds holds at least
// blockDim.x / 64 doubles.
__device__ double block_reduce(double v, double *lds) {
  v = wave_sum_dpp(v);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  for (int w = 0; w < int(blockDim.x >> 6); ++w) r += lds[w];
  __syncthreads();
  return r;
}

// sum of count partials, identical in every thread of the block (fixed order)
__device__ double block_sum(const double *part, int64_t count, int stride, double *lds) {
  double s = 0.0;
  for (int64_t k = threadIdx.x; k < count; k += blockDim.x) s += part[k * stride];
  return block_reduce(s, lds);
}

__device__ __forceinline__ bool finite(double x) { return isfinite(x); }

// ---- statistics -----------------------------------------------------------------
template <bool C>
__device__ __forceinline__ void k_sum_e_body(int BX, int BY, int BZ, int GX, int64_t n, const double *e, double *part) {
  __shared__ double lds[256];
  const int64_t s = int64_t(BX) * 256 + threadIdx.x;
  double r = 0.0, i = 0.0;
  if (s < n) {
    r = C ? e[2 * s] : e[s];
    i = C ? e[2 * s + 1] : 0.0;
  }
  r = block_reduce(r, lds);
  i = block_reduce(i, lds);
  if (threadIdx.x == 0) {
    part[2 * BX] = r;
    part[2 * BX + 1] = i;
  }
}

template <bool C>
__global__ __launch_bounds__(256) void k_sum_e(int64_t n, const double *e, double *part) {
  k_sum_e_body<C>(blockIdx.x, blockIdx.y, blockIdx.z, gridDim.x, n, e, part);
}

// u_s = E_s - E (E from the partials), per-block partial sums of |u|^2
template <bool C>
__device__ __forceinline__ void k_center_e_body(int BX, int BY, int BZ, int GX, int64_t n, const double *e,
                                                   const double *part, int64_t nparts,
                                                   double *u, double *part2, CGState *st) {
  __shared__ double lds[256];
  const double Er = block_sum(part, nparts, 2, lds) / double(n);
  const double Ei = block_sum(part + 1, nparts, 2, lds) / double(n);
  if (BX == 0 && threadIdx.x == 0) {
    st->E[0] = Er;
    st->E[1] = Ei;
  }
  const int64_t s = int64_t(BX) * 256 + threadIdx.x;
  double v = 0.0;
  if (s < n) {
    double ur = (C ? e[2 * s] : e[s]) - Er;
    double ui = C ? e[2 * s + 1] - Ei : 0.0;
    if (C) {
      u[2 * s] = ur;
      u[2 * s + 1] = ui;
    } else {
      u[s] = ur;
    }
    v = ur * ur + ui * ui;
  }
  v = block_reduce(v, lds);
  if (threadIdx.x == 0) part2[BX] = v;
}

template <bool C>
__global__ __launch_bounds__(256) void k_center_e(int64_t n, const double *e,
                                                   const double *part, int64_t nparts,
                                                   double *u, double *part2, CGState *st) {
  k_center_e_body<C>(blockIdx.x, blockIdx.y, blockIdx.z, gridDim.x, n, e, part, nparts, u, part2, st);
}

// ---- error bar of the energy (chain means) -----------------------------------------
// Samples are laid out [S sweeps, nch chains]. Block BX takes chains 64 BX .. 64 BX + 63:
// thread t sums chain 64 BX + (t & 63) over the sweeps q = t / 64 (mod 4), four slices
// combined in a fixed order; cm[c] = mean over the sweeps of Re E_loc; per-block partial
// sums of the chain means follow.
constexpr int kChainsPerBlock = 64;
template <bool C>
__device__ __forceinline__ void k_chain_mean_body(int BX, int64_t n, int64_t nch,
                                                  const double *e, double *cm,
                                                  double *cpart) {
  __shared__ double lds[256];
  __shared__ double sl[4][kChainsPerBlock];
  const int64_t S = n / nch;
  const int ch = threadIdx.x & 63, q0 = threadIdx.x >> 6;
  const int64_t c = int64_t(BX) * kChainsPerBlock + ch;
  double s0 = 0.0, s1 = 0.0;
  if (c < nch) {
    int64_t q = q0;
    for (; q + 4 < S; q += 8) {
      s0 += C ? e[2 * (q * nch + c)] : e[q * nch + c];
      s1 += C ? e[2 * ((q + 4) * nch + c)] : e[(q + 4) * nch + c];
    }
    if (q < S) s0 += C ? e[2 * (q * nch + c)] : e[q * nch + c];
  }
  sl[q0][ch] = s0 + s1;
  __syncthreads();
  double m = 0.0;
  if (q0 == 0 && c < nch) {
    m = (((sl[0][ch] + sl[1][ch]) + sl[2][ch]) + sl[3][ch]) / double(S);
    cm[c] = m;
  }
  m = block_reduce(m, lds);
  if (threadIdx.x == 0) cpart[BX] = m;
}

template <bool C>
__global__ __launch_bounds__(256) void k_chain_mean(int64_t n, int64_t nch, const double *e,
                                                    double *cm, double *cpart) {
  k_chain_mean_body<C>(blockIdx.x, n, nch, e, cm, cpart);
}

// per-block partial sums of (m_c - mean m)^2 (the mean from the partials, in every block)
__device__ __forceinline__ void k_chain_dev_body(int BX, int64_t nch, const double *cm,
                                                 const double *cpart, int64_t ncb,
                                                 double *cpart2) {
  __shared__ double lds[256];
  const double mbar = block_sum(cpart, ncb, 1, lds) / double(nch);
  const int64_t c = int64_t(BX) * 256 + threadIdx.x;
  double d = 0.0;
  if (c < nch) {
    d = cm[c] - mbar;
    d *= d;
  }
  d = block_reduce(d, lds);
  if (threadIdx.x == 0) cpart2[BX] = d;
}

__global__ __launch_bounds__(256) void k_chain_dev(int64_t nch, const double *cm,
                                                   const double *cpart, int64_t ncb,
                                                   double *cpart2) {
  k_chain_dev_body(blockIdx.x, nch, cm, cpart, ncb, cpart2);
}

__global__ void k_fill(int64_t count, double *x, double val) {
  for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < count;
       k += int64_t(gridDim.x) * blockDim.x)
    x[k] = val;
}

// write the CG direction p (complex double, packed like the parameters) as the tables the
// product kernels read: Vt[i][j] = p_W[j][i], vb = p_b (compute precision), va = p_a
template <typename T, bool C>
__device__ __forceinline__ void dir_write(int N, int M, int64_t k, double pr, double pi, T *Vt,
                                          T *vb, double *va, int split) {
  if (k < N) {
    va[2 * k] = pr;
    va[2 * k + 1] = pi;
  } else if (k < N + M) {
    vstore<T, C>(vb, k - N, vmake<T, C>(T(pr), T(pi)));
  } else {
    const int64_t q = k - N - M;
    vstore<T, C>(Vt, (q % N) * M + q / N, vmake<T, C>(T(pr), T(pi)));
    if (sizeof(T) == 4 && split) {
      // the bf16 split that follows V^T (the JVP's operand on the bf16 matrix cores)
      uint16_t *Vs = reinterpret_cast<uint16_t *>(reinterpret_cast<char *>(Vt) +
                                                  vsplit_offset(N, M, sizeof(T) * (C ? 2 : 1)));
      vsplit_store<C>(Vs, N, M, int(q % N), int(q / N), float(pr), float(pi));
    }
  }
}

// zero the padding sites [N, Np8) of the split direction (FP32 tables)
template <typename T, bool C>
__device__ __forceinline__ void dir_pad_zero(int N, int M, int64_t first, int64_t stride, T *Vt) {
  if constexpr (sizeof(T) == 4) {
    const int np = vsplit_np8(N);
    if (np == N) return;
    uint16_t *Vs = reinterpret_cast<uint16_t *>(reinterpret_cast<char *>(Vt) +
                                                vsplit_offset(N, M, sizeof(T) * (C ? 2 : 1)));
    const int64_t pad = int64_t(C ? 2 : 1) * 3 * M * (np - N);
    for (int64_t q = first; q < pad; q += stride) {
      const int i = N + int(q % (np - N));
      const int64_t r = q / (np - N);
      const int64_t pp = r / M, j = r % M;
      Vs[((pp * (np / 8) + i / 8) * M + j) * 8 + i % 8] = 0;
    }
  }
}

// variance; F = g / n; x = 0; r = p = F (+ direction tables); partial ||F||^2
template <typename T, bool C>
__device__ __forceinline__ void k_cg_init_body(int BX, int BY, int BZ, int GX, int N, int M, int64_t n, const double *part2,
                                                  int64_t nparts, const double *g, double *F,
                                                  double *x, double *r, double *p, T *Vt, T *vb,
                                                  double *va, double *dpart, CGState *st,
    int split) {
  __shared__ double lds[256];
  const int64_t P = int64_t(N) + M + int64_t(N) * M;
  if (BX == 0) {
    double var = block_sum(part2, nparts, 1, lds) / double(n);
    if (threadIdx.x == 0) st->var = var;
  }
  double acc = 0.0;
  for (int64_t k = int64_t(BX) * 256 + threadIdx.x; k < P;
       k += int64_t(GX) * 256) {
    const double fr = (C ? g[2 * k] : g[k]) / double(n);
    const double fi = C ? g[2 * k + 1] / double(n) : 0.0;
    if (C) {
      F[2 * k] = fr;
      F[2 * k + 1] = fi;
      x[2 * k] = 0.0;
      x[2 * k + 1] = 0.0;
      r[2 * k] = fr;
      r[2 * k + 1] = fi;
      p[2 * k] = fr;
      p[2 * k + 1] = fi;
    } else {
      F[k] = fr;
      x[k] = 0.0;
      r[k] = fr;
      p[k] = fr;
    }
    dir_write<T, C>(N, M, k, fr, fi, Vt, vb, va, split);
    acc += fr * fr + fi * fi;
  }
  if (split) dir_pad_zero<T, C>(N, M, int64_t(BX) * 256 + threadIdx.x, int64_t(GX) * 256, Vt);
  acc = block_reduce(acc, lds);
  if (threadIdx.x == 0) dpart[BX] = acc;
}

template <typename T, bool C>
__global__ __launch_bounds__(256) void k_cg_init(int N, int M, int64_t n, const double *part2,
                                                  int64_t nparts, const double *g, double *F,
                                                  double *x, double *r, double *p, T *Vt, T *vb,
                                                  double *va, double *dpart, CGState *st,
    int split) {
  k_cg_init_body<T, C>(blockIdx.x, blockIdx.y, blockIdx.z, gridDim.x, N, M, n, part2, nparts, g, F, x, r, p, Vt, vb, va, dpart, st, split);
}

__device__ __forceinline__ void k_cg_start_body(int BX, int BY, int BZ, int GX, const double *dpart, int64_t nparts,
                                                  double tol, int maxiter, CGState *st,
                                                  const double *cpart2, int64_t ncb2,
                                                  int64_t nch) {
  __shared__ double lds[256];
  double rr = block_sum(dpart, nparts, 1, lds);
  const double dev2 = block_sum(cpart2, ncb2, 1, lds);
  if (threadIdx.x == 0) {
    st->err = sqrt(dev2 / double(nch - 1)) / sqrt(double(nch));
    st->rr[0] = rr;
    st->rr[1] = rr;
    st->bnorm = sqrt(rr);
    st->fnorm = sqrt(rr);
    st->iters = 0;
    st->alpha = 0.0;
    st->converged = 0;
    st->nonfinite = !(finite(rr) && finite(st->E[0]) && finite(st->E[1]) && finite(st->var));
    st->done = st->nonfinite || rr == 0.0 || maxiter <= 0;
    if (rr == 0.0) st->converged = 1;
  }
}

__global__ __launch_bounds__(256) void k_cg_start(const double *dpart, int64_t nparts,
                                                  double tol, int maxiter, CGState *st,
                                                  const double *cpart2, int64_t ncb2,
                                                  int64_t nch) {
  k_cg_start_body(blockIdx.x, blockIdx.y, blockIdx.z, gridDim.x, dpart, nparts, tol, maxiter, st,
                  cpart2, ncb2, nch);
}

// g = O^dagger y from the first-level sums, then
// Ap = (g - ybar * O^dagger 1) / n + lambda p ; partial Re(p^dagger Ap)
template <bool C>
__device__ __forceinline__ void k_cg_ap_body(int BX, int BY, int BZ, int GX, int N, int M, int64_t n, int groups, int colsP,
                                               int64_t elems, const double *out1,
                                               const double *o1, const double *ysum,
                                               int64_t nys, const double *p, double lambda,
                                               double *Ap, double *dpart, const CGState *st) {
  if (st->done) return;
  __shared__ double lds[256];
  const int64_t P = int64_t(N) + M + int64_t(N) * M;
  const double ybr = block_sum(ysum, nys, 2, lds) / double(n);
  const double ybi = C ? block_sum(ysum + 1, nys, 2, lds) / double(n) : 0.0;
  double acc = 0.0;
  for (int64_t k = int64_t(BX) * 256 + threadIdx.x; k < P;
       k += int64_t(GX) * 256) {
    int64_t e;
    if (k < N)
      e = int64_t(M) * colsP + k;
    else if (k < N + M)
      e = int64_t(k - N) * colsP + N;
    else
      e = ((k - N - M) / N) * colsP + ((k - N - M) % N);
    double gr = 0.0, gi = 0.0;
    for (int q = 0; q < groups; ++q) {
      gr += out1[2 * (int64_t(q) * elems + e)];
      gi += out1[2 * (int64_t(q) * elems + e) + 1];
    }
    if (C) {
      gr -= ybr * o1[2 * k] - ybi * o1[2 * k + 1];
      gi -= ybr * o1[2 * k + 1] + ybi * o1[2 * k];
      const double ar = gr / double(n) + lambda * p[2 * k];
      const double ai = gi / double(n) + lambda * p[2 * k + 1];
      Ap[2 * k] = ar;
      Ap[2 * k + 1] = ai;
      acc += p[2 * k] * ar + p[2 * k + 1] * ai;
    } else {
      const double ar = (gr - ybr * o1[k]) / double(n) + lambda * p[k];
      Ap[k] = ar;
      acc += p[k] * ar;
    }
  }
  acc = block_reduce(acc, lds);
  if (threadIdx.x == 0) dpart[BX] = acc;
}

template <bool C>
__global__ __launch_bounds__(256) void k_cg_ap(int N, int M, int64_t n, int groups, int colsP,
                                               int64_t elems, const double *out1,
                                               const double *o1, const double *ysum,
                                               int64_t nys, const double *p, double lambda,
                                               double *Ap, double *dpart, const CGState *st) {
  k_cg_ap_body<C>(blockIdx.x, blockIdx.y, blockIdx.z, gridDim.x, N, M, n, groups, colsP, elems, out1, o1, ysum, nys, p, lambda, Ap, dpart, st);
}

// alpha = rr / p^dagger Ap ; x += alpha p ; r -= alpha Ap ; partial r^dagger r
__device__ __forceinline__ void k_cg_xr_body(int BX, int BY, int BZ, int GX, int64_t Pc, const double *dpart, int64_t nparts,
                                               int parity, double *x, double *r,
                                               const double *p, const double *Ap,
                                               double *rpart, CGState *st) {
  if (st->done) return;
  __shared__ double lds[256];
  const double pAp = block_sum(dpart, nparts, 1, lds);
  const double alpha = st->rr[parity] / pAp;
  double acc = 0.0;
  for (int64_t k = int64_t(BX) * 256 + threadIdx.x; k < Pc;
       k += int64_t(GX) * 256) {
    x[k] += alpha * p[k];
    double rk = r[k] - alpha * Ap[k];
    r[k] = rk;
    acc += rk * rk;
  }
  acc = block_reduce(acc, lds);
  if (threadIdx.x == 0) rpart[BX] = acc;
  if (BX == 0 && threadIdx.x == 0) st->alpha = alpha;
}

__global__ __launch_bounds__(256) void k_cg_xr(int64_t Pc, const double *dpart, int64_t nparts,
                                               int parity, double *x, double *r,
                                               const double *p, const double *Ap,
                                               double *rpart, CGState *st) {
  k_cg_xr_body(blockIdx.x, blockIdx.y, blockIdx.z, gridDim.x, Pc, dpart, nparts, parity, x, r, p, Ap, rpart, st);
}

// the sum of a CG step's block partials, once, in a fixed order (1024 threads, four
// independent strided sums each, then a tree): the consumers then read a single partial
__global__ __launch_bounds__(1024) void k_psum(const double *part, int64_t nparts, double *out,
                                               const CGState *st) {
  if (st->done) return;
  __shared__ double lds[1024];
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int64_t k = threadIdx.x;
  for (; k + 3 * 1024 < nparts; k += 4 * 1024) {
    a0 += part[k];
    a1 += part[k + 1024];
    a2 += part[k + 2 * 1024];
    a3 += part[k + 3 * 1024];
  }
  for (; k < nparts; k += 1024) a0 += part[k];
  lds[threadIdx.x] = (a0 + a1) + (a2 + a3);
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (threadIdx.x < w) lds[threadIdx.x] += lds[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = lds[0];
}

// rr_new from partials; convergence; beta = rr_new / rr ; p = r + beta p (+ direction
// tables for the next product)
template <typename T, bool C>
__device__ __forceinline__ void k_cg_p_body(int BX, int BY, int BZ, int GX, int N, int M, const double *rpart, int64_t nparts,
                                              int parity, double tol, int maxiter,
                                              const double *r, double *p, T *Vt, T *vb,
                                              double *va, CGState *st,
    int split) {
  if (st->done) return;
  __shared__ double lds[256];
  const int64_t P = int64_t(N) + M + int64_t(N) * M;
  const double rr_new = block_sum(rpart, nparts, 1, lds);
  const double rr = st->rr[parity];
  const double beta = rr_new / rr;
  const int iters = st->iters + 1;
  const bool conv = sqrt(rr_new) <= tol * st->bnorm;
  const bool bad = !(finite(rr_new) && finite(st->alpha));
  auto update = [&](int64_t k) __attribute__((always_inline)) {
    double pr, pi = 0.0;
    if (C) {
      pr = r[2 * k] + beta * p[2 * k];
      pi = r[2 * k + 1] + beta * p[2 * k + 1];
      p[2 * k] = pr;
      p[2 * k + 1] = pi;
    } else {
      pr = r[k] + beta * p[k];
      p[k] = pr;
    }
    dir_write<T, C>(N, M, k, pr, pi, Vt, vb, va, split);
  };
  // a and b in parameter order
  for (int64_t k = int64_t(BX) * 256 + threadIdx.x; k < N + M; k += int64_t(GX) * 256)
    update(k);
  // W in tiles of 8 sites x 8 hidden units per 64 threads (site fastest): the reads of r
  // and p and the writes of V^T and of its bf16 split all cover whole 64- or 128-byte
  // runs (parameter order alone would scatter the transposed writes)
  const int tN = (N + 7) >> 3;
  const int64_t nt = int64_t(tN) * ((M + 7) >> 3) * 64;
  for (int64_t g = int64_t(BX) * 256 + threadIdx.x; g < nt; g += int64_t(GX) * 256) {
    const int64_t tile = g >> 6;
    const int lane = int(g & 63);
    const int i = int(tile % tN) * 8 + (lane & 7);
    const int j = int(tile / tN) * 8 + (lane >> 3);
    if (i < N && j < M) update(int64_t(N) + M + int64_t(j) * N + i);
  }
  __syncthreads();
  if (BX == 0 && threadIdx.x == 0) {
    st->rr[parity ^ 1] = rr_new;
    st->iters = iters;
    st->converged = conv;
    st->nonfinite = bad;
    st->done = conv || bad || iters >= maxiter;
  }
}

template <typename T, bool C>
__global__ __launch_bounds__(256) void k_cg_p(int N, int M, const double *rpart, int64_t nparts,
                                              int parity, double tol, int maxiter,
                                              const double *r, double *p, T *Vt, T *vb,
                                              double *va, CGState *st,
    int split) {
  k_cg_p_body<T, C>(blockIdx.x, blockIdx.y, blockIdx.z, gridDim.x, N, M, rpart, nparts, parity, tol, maxiter, r, p, Vt, vb, va, st, split);
}

// ---- fused CG iteration kernel (single model) -----------------------------------
// g = sum over the sample splits of the VJP partial tiles, then
// Ap = (g - ybar O^dagger 1) / n + lambda p and per-block partial sums of Re(p^dagger Ap).
// A block takes 32 elements of the tile layout; its 8 thread slices sum every eighth
// split of them, and the slices are added in a fixed order (deterministic). Elements
// outside the parameters are idle.
// SL slices of 256 / SL elements per block: 8 slices (32 elements) when there are many
// sample splits to add, one slice (256 elements) when there are few
constexpr int kAprElems = 32;
inline int apr_slices(int splits) { return splits >= 8 ? 8 : 1; }
inline int64_t apr_blocks(int64_t elems, int splits) {
  return (elems + 256 / apr_slices(splits) - 1) / (256 / apr_slices(splits));
}

template <typename T, bool C, int SL>
__global__ __launch_bounds__(256) void k_cg_apr_t(int N, int M, int64_t n, int splits,
                                                int colsP, int64_t elems,
                                                const T *__restrict__ part,
                                                const double *o1, const double *ysum,
                                                int64_t nys, const double *p, double lambda,
                                                double *Ap, double *dpart, const CGState *st) {
  __shared__ double lds[256];
  constexpr int kE = 256 / SL;
  __shared__ double sr[SL][kE], si[SL][kE];
  // the solver state and the sums of y in one memory round trip (no state: a single
  // product, always computed)
  const int done = st ? st->done : 0;
  double ysr = 0.0, ysi = 0.0;
  for (int64_t k = threadIdx.x; k < nys; k += blockDim.x) {
    ysr += ysum[2 * k];
    if (C) ysi += ysum[2 * k + 1];
  }
  if (done) return;
  const int el = threadIdx.x % kE, sl = threadIdx.x / kE;
  const int64_t e = int64_t(blockIdx.x) * kE + el;
  // parameter index of the element (-1: padding of the tile layout)
  int64_t k = -1;
  if (e < elems) {
    const int jrow = int(e / colsP), icol = int(e % colsP);
    if (jrow < M && icol < N)
      k = int64_t(N) + M + int64_t(jrow) * N + icol;  // W_ji
    else if (jrow < M && icol == N)
      k = N + jrow;  // b_j
    else if (jrow == M && icol < N)
      k = icol;  // a_i
  }
  // the direction and O^dagger 1 of the element, loaded with the partial tiles
  double pr = 0.0, pim = 0.0, o1r = 0.0, o1i = 0.0;
  if (sl == 0 && k >= 0) {
    pr = p[C ? 2 * k : k];
    o1r = o1[C ? 2 * k : k];
    if (C) {
      pim = p[2 * k + 1];
      o1i = o1[2 * k + 1];
    }
  }
  double gr = 0.0, gi = 0.0;
  if (k >= 0) {
    // up to 32 loads in flight per thread, added in split order (padding entries of the
    // tile layout are not read)
    int q = sl;
    for (; q + 31 * SL < splits; q += 32 * SL) {
      V<T, C> xs[32];
#pragma unroll
      for (int u = 0; u < 32; ++u) xs[u] = vload<T, C>(part, int64_t(q + u * SL) * elems + e);
#pragma unroll
      for (int u = 0; u < 32; ++u) {
        gr += double(xs[u].re);
        if (C) gi += double(xs[u].im);
      }
    }
    for (; q + 7 * SL < splits; q += 8 * SL) {
      V<T, C> xs[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) xs[u] = vload<T, C>(part, int64_t(q + u * SL) * elems + e);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        gr += double(xs[u].re);
        if (C) gi += double(xs[u].im);
      }
    }
    for (; q < splits; q += SL) {
      const V<T, C> x = vload<T, C>(part, int64_t(q) * elems + e);
      gr += double(x.re);
      if (C) gi += double(x.im);
    }
  }
  const double ybr = block_reduce(ysr, lds) / double(n);
  const double ybi = C ? block_reduce(ysi, lds) / double(n) : 0.0;
  sr[sl][el] = gr;
  si[sl][el] = gi;
  __syncthreads();
  double acc = 0.0;
  if (sl == 0 && k >= 0) {
    for (int q = 1; q < SL; ++q) {
      gr += sr[q][el];
      gi += si[q][el];
    }
    if (C) {
      gr -= ybr * o1r - ybi * o1i;
      gi -= ybr * o1i + ybi * o1r;
      const double ar = gr / double(n) + lambda * pr;
      const double ai = gi / double(n) + lambda * pim;
      Ap[2 * k] = ar;
      Ap[2 * k + 1] = ai;
      acc = pr * ar + pim * ai;
    } else {
      const double ar = (gr - ybr * o1r) / double(n) + lambda * pr;
      Ap[k] = ar;
      acc = pr * ar;
    }
  }
  acc = block_reduce(acc, lds);
  if (threadIdx.x == 0) dpart[blockIdx.x] = acc;
}

// launch of the CG product reduction with the slice count of the split count
template <typename T, bool C>
void k_cg_apr_launch(int64_t elems, hipStream_t st, int N, int M, int64_t n, int splits,
                     int colsP, const T *part, const double *o1, const double *ysum, int64_t nys,
                     const double *p, double lambda, double *Ap, double *dpart,
                     const CGState *state) {
  const dim3 grid(unsigned(apr_blocks(elems, splits)));
  if (apr_slices(splits) == 8)
    hipLaunchKernelGGL((k_cg_apr_t<T, C, 8>), grid, dim3(256), 0, st, N, M, n, splits, colsP,
                       elems, part, o1, ysum, nys, p, lambda, Ap, dpart, state);
  else
    hipLaunchKernelGGL((k_cg_apr_t<T, C, 1>), grid, dim3(256), 0, st, N, M, n, splits, colsP,
                       elems, part, o1, ysum, nys, p, lambda, Ap, dpart, state);
}

// ---- x, r and p of one CG iteration in one block (small parameter counts) ----------
// alpha = rr / p^dagger Ap; x += alpha p; r -= alpha Ap; rr_new = r^dagger r;
// beta = rr_new / rr; p = r + beta p (+ direction tables). Thread t owns elements
// t + kXrpThreads i (i < kXrpPer): all their loads are issued before the sum of p^dagger Ap
// is formed, and the values stay in registers between the two passes.
constexpr int kXrpThreads = 1024;
constexpr int kXrpPer = 4;
constexpr int64_t kXrpMaxParams = int64_t(kXrpThreads) * kXrpPer;

template <typename T, bool C>
__global__ __launch_bounds__(kXrpThreads) void k_cg_xrp(int N, int M, const double *dpart,
                                                        int64_t nparts, int parity, double tol,
                                                        int maxiter, double *x, double *r,
                                                        double *p, const double *Ap, T *Vt,
                                                        T *vb, double *va, CGState *st,
    int split) {
  __shared__ double lds[kXrpThreads / 64];
  constexpr int cs = C ? 2 : 1;
  const int64_t P = int64_t(N) + M + int64_t(N) * M;
  // the solver state is read together with the vectors (one memory round trip); a
  // finished solve returns after the loads
  const int done = st->done;
  const double rr = st->rr[parity], bnorm = st->bnorm;
  const int iters0 = st->iters;
  double xv[kXrpPer][cs], rv[kXrpPer][cs], pv[kXrpPer][cs], av[kXrpPer][cs];
#pragma unroll
  for (int i = 0; i < kXrpPer; ++i) {
    const int64_t k = threadIdx.x + int64_t(kXrpThreads) * i;
    const int64_t kk = k < P ? k : 0;
#pragma unroll
    for (int c = 0; c < cs; ++c) {
      xv[i][c] = x[cs * kk + c];
      rv[i][c] = r[cs * kk + c];
      pv[i][c] = p[cs * kk + c];
      av[i][c] = Ap[cs * kk + c];
    }
  }
  double pa = 0.0;
  for (int64_t k = threadIdx.x; k < nparts; k += kXrpThreads) pa += dpart[k];
  if (done) return;
  const double pAp = block_reduce(pa, lds);
  const double alpha = rr / pAp;
  double acc = 0.0;
#pragma unroll
  for (int i = 0; i < kXrpPer; ++i) {
    const int64_t k = threadIdx.x + int64_t(kXrpThreads) * i;
    if (k < P) {
#pragma unroll
      for (int c = 0; c < cs; ++c) {
        xv[i][c] += alpha * pv[i][c];
        rv[i][c] -= alpha * av[i][c];
        x[cs * k + c] = xv[i][c];
        r[cs * k + c] = rv[i][c];
        acc += rv[i][c] * rv[i][c];
      }
    }
  }
  const double rr_new = block_reduce(acc, lds);
  const double beta = rr_new / rr;
#pragma unroll
  for (int i = 0; i < kXrpPer; ++i) {
    const int64_t k = threadIdx.x + int64_t(kXrpThreads) * i;
    if (k < P) {
      const double pr = rv[i][0] + beta * pv[i][0];
      const double pi = C ? rv[i][cs - 1] + beta * pv[i][cs - 1] : 0.0;
      p[cs * k] = pr;
      if (C) p[cs * k + cs - 1] = pi;
      dir_write<T, C>(N, M, k, pr, pi, Vt, vb, va, split);
    }
  }
  if (threadIdx.x == 0) {
    const int iters = iters0 + 1;
    const bool conv = sqrt(rr_new) <= tol * bnorm;
    const bool bad = !(finite(rr_new) && finite(alpha));
    st->alpha = alpha;
    st->rr[parity ^ 1] = rr_new;
    st->iters = iters;
    st->converged = conv;
    st->nonfinite = bad;
    st->done = conv || bad || iters >= maxiter;
  }
}

// whether the step's energy, variance and every CG scalar are finite
__device__ __forceinline__ bool step_finite(const CGState *st) {
  return !st->nonfinite && finite(st->E[0]) && finite(st->E[1]) && finite(st->var);
}

template <typename PT>
__device__ __forceinline__ void k_update_body(int BX, int BY, int BZ, int GX, int64_t Pc, PT *params, const double *x, double lr) {
  for (int64_t k = BX * int64_t(blockDim.x) + threadIdx.x; k < Pc;
       k += int64_t(GX) * blockDim.x)
    params[k] = PT(double(params[k]) - lr * x[k]);
}

// p <- p - lr x, only when the step is finite (decided on the device)
template <typename PT>
__global__ void k_update(int64_t Pc, PT *params, const double *x, double lr,
                         const CGState *st) {
  if (!step_finite(st)) return;
  k_update_body<PT>(blockIdx.x, blockIdx.y, blockIdx.z, gridDim.x, Pc, params, x, lr);
}

__device__ __host__ inline void fill_info(const CGState &h, nqs_sr_info *o) {
  const bool nf = h.nonfinite || !isfinite(h.E[0]) || !isfinite(h.E[1]) || !isfinite(h.var);
  o->cg_iters = h.iters;
  o->converged = h.converged;
  o->cg_resid = h.bnorm > 0 ? sqrt(h.rr[h.iters & 1]) / h.bnorm : 0.0;
  o->energy_re = h.E[0];
  o->energy_im = h.E[1];
  o->variance = h.var;
  o->force_norm = h.fnorm;
  o->energy_err = h.err;
  o->status = nf ? NQS_ENONFINITE : (h.converged ? NQS_OK : NQS_ENOTCONV);
  o->reserved = 0;
}

// the step's information, written to device memory in stream order
__global__ void k_sr_info(const CGState *st, nqs_sr_info *out) {
  if (threadIdx.x == 0) fill_info(*st, out);
}

struct SRLayout {
  size_t grad, y, ysum, u, e_part, e_part2, cm, c_part, c_part2, o1, g, F, x, r, p, Ap, dpart,
      rpart, vexp, apexp, o1s, gs, ybar, psum, state, total;
};

SRLayout sr_layout(const nqs_model *m, int64_t n) {
  const int cs = m->is_complex ? 2 : 1;
  const bool ff = m->ff.L > 0;
  const int64_t P = ff ? m->ff.P : int64_t(m->N) + m->M + int64_t(m->N) * m->M;
  const int64_t nb = cdiv(n, 256);
  const int64_t pb = cdiv(P, 256) < 4096 ? cdiv(P, 256) : 4096;
  SRLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += (bytes + 255) / 256 * 256;
    return o;
  };
  L.grad = take(ff ? ff_grad_scratch_bytes(m, n) : grad_scratch_bytes(m, n));
  L.y = take(size_t(n) * cs * 8);
  const int64_t ns = ff ? ff_jvp_blocks(m, n) : grad_plan(m, n).splits;
  const int64_t ncap = ns > 2 * int64_t(m->cu_count) ? ns : 2 * int64_t(m->cu_count);
  L.ysum = take(size_t(nb > ncap ? nb : ncap) * 16);
  L.u = take(size_t(n) * cs * 8);
  L.e_part = take(size_t(nb) * 16);
  L.e_part2 = take(size_t(nb) * 8);
  L.cm = take(size_t(n) * 8);
  L.c_part = take(size_t(cdiv(n, kChainsPerBlock)) * 8);
  L.c_part2 = take(size_t(nb) * 8);
  L.o1 = take(size_t(P) * cs * 8);
  L.g = take(size_t(P) * cs * 8);
  L.F = take(size_t(P) * cs * 8);
  L.x = take(size_t(P) * cs * 8);
  L.r = take(size_t(P) * cs * 8);
  L.p = take(size_t(P) * cs * 8);
  L.Ap = take(size_t(P) * cs * 8);
  {
    // partial sums of p^dagger Ap: per block of the parameter range, or of the VJP tile
    // layout (k_cg_apr), whichever has more blocks
    const GradPlan gq = grad_plan(m, n);
    const int64_t ab = ff ? 0 : cdiv(int64_t(gq.Jtiles) * 16 * gq.Itiles * 16, kAprElems);
    L.dpart = take(size_t(pb > ab ? pb : ab) * 8);
  }
  const int64_t cb = cdiv(P * cs, 256) < 4096 ? cdiv(P * cs, 256) : 4096;
  L.rpart = take(size_t(cb) * 8);
  // symmetric RBM: the expanded direction and product, O^dagger 1 and the force numerator
  // in the symmetric parameters (the CG vectors above hold the symmetric ones)
  const size_t se = m->G ? size_t(P) * cs * 8 : 0;
  const size_t ss = m->G ? size_t(n_params_model(m)) * cs * 8 : 0;
  L.vexp = take(se);
  L.apexp = take(se);
  L.o1s = take(ss);
  L.gs = take(ss);
  L.ybar = take(16);
  L.psum = take(16);
  L.state = take(sizeof(CGState));
  L.total = off;
  return L;
}

#define HIPTRY(x)                             \
  do {                                        \
    hipError_t e__ = (x);                     \
    if (e__ != hipSuccess) return NQS_EDEVICE; \
  } while (0)

template <bool C>
__device__ __forceinline__ void k_ones_body(int BX, int BY, int BZ, int GX, int64_t n, double *u) {
  for (int64_t s = BX * int64_t(blockDim.x) + threadIdx.x; s < n;
       s += int64_t(GX) * blockDim.x) {
    if (C) {
      u[2 * s] = 1.0;
      u[2 * s + 1] = 0.0;
    } else {
      u[s] = 1.0;
    }
  }
}

template <bool C>
__global__ void k_ones(int64_t n, double *u) {
  k_ones_body<C>(blockIdx.x, blockIdx.y, blockIdx.z, gridDim.x, n, u);
}

inline unsigned grid_for(int64_t count) {
  int64_t b = cdiv(count, 256);
  return unsigned(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

// ---- symmetric RBM: CG in the symmetric parameters --------------------------------------
// F = g / n; x = 0; r = p = F; variance; partials of ||F||^2 (no direction tables: the
// direction is expanded before every product)
template <bool C>
__global__ __launch_bounds__(256) void k_symm_cg_init(int64_t Ps, int64_t n, const double *part2,
                                                      int64_t nparts, const double *g, double *F,
                                                      double *x, double *r, double *p,
                                                      double *dpart, CGState *st) {
  __shared__ double lds[256];
  constexpr int cs = C ? 2 : 1;
  if (blockIdx.x == 0) {
    const double var = block_sum(part2, nparts, 1, lds) / double(n);
    if (threadIdx.x == 0) st->var = var;
  }
  double acc = 0.0;
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < Ps; k += int64_t(gridDim.x) * 256) {
#pragma unroll
    for (int c = 0; c < cs; ++c) {
      const double f = g[cs * k + c] / double(n);
      F[cs * k + c] = f;
      x[cs * k + c] = 0.0;
      r[cs * k + c] = f;
      p[cs * k + c] = f;
      acc += f * f;
    }
  }
  acc = block_reduce(acc, lds);
  if (threadIdx.x == 0) dpart[blockIdx.x] = acc;
}

// Ap += lambda p on the reduced product; partials of Re(p^dagger Ap)
__global__ __launch_bounds__(256) void k_symm_shift_dot(int64_t Pc, const double *p,
                                                        double lambda, double *Ap, double *dpart,
                                                        const CGState *st) {
  if (st && st->done) return;
  __shared__ double lds[256];
  double acc = 0.0;
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < Pc; k += int64_t(gridDim.x) * 256) {
    const double a = Ap[k] + lambda * p[k];
    Ap[k] = a;
    acc += p[k] * a;
  }
  acc = block_reduce(acc, lds);
  if (threadIdx.x == 0 && dpart) dpart[blockIdx.x] = acc;
}

// rr_new from partials; convergence; beta = rr_new / rr; p = r + beta p (no tables)
__global__ __launch_bounds__(256) void k_cg_p_plain(int64_t Pc, const double *rpart,
                                                    int64_t nparts, int parity, double tol,
                                                    int maxiter, const double *r, double *p,
                                                    CGState *st) {
  if (st->done) return;
  __shared__ double lds[256];
  const double rr_new = block_sum(rpart, nparts, 1, lds);
  const double beta = rr_new / st->rr[parity];
  const int iters = st->iters + 1;
  const bool conv = sqrt(rr_new) <= tol * st->bnorm;
  const bool bad = !(finite(rr_new) && finite(st->alpha));
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < Pc; k += int64_t(gridDim.x) * 256)
    p[k] = r[k] + beta * p[k];
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->rr[parity ^ 1] = rr_new;
    st->iters = iters;
    st->converged = conv;
    st->nonfinite = bad;
    st->done = conv || bad || iters >= maxiter;
  }
}

// async: queue cg_maxiter iteration slots and write the information to device memory
// (info is then a device pointer); otherwise check convergence on the host between
// chunks and fill the host struct info
template <typename T, bool C>
nqs_status sr_impl(nqs_model *m, void *params, const int8_t *sigma, const void *eloc,
                   int64_t n, int64_t nch, double lr, double diag_shift, double cg_tol,
                   int cg_maxiter, void *ws, nqs_sr_info *info, bool async, hipStream_t st) {
  SRLayout L = sr_layout(m, n);
  char *b = (char *)ws;
  auto D = [&](size_t off) { return (double *)(b + off); };
  CGState *state = (CGState *)(b + L.state);
  void *grad = b + L.grad;
  const int cs = C ? 2 : 1;
  const int N = m->N, M = m->M;
  const int64_t P = int64_t(N) + M + int64_t(N) * M;
  const int64_t Pc = P * cs;
  const int64_t nb = cdiv(n, 256);
  const int64_t pblocks = cdiv(P, 256) < 4096 ? cdiv(P, 256) : 4096;
  const int64_t cblocks = cdiv(Pc, 256) < 4096 ? cdiv(Pc, 256) : 4096;
  const GradPlan gp = grad_plan(m, n);
  const GradBuffers gb = grad_buffers(m, n, grad);
  const int64_t elems = int64_t(gp.Jtiles) * 16 * gp.Itiles * 16;
  const int64_t nys = gp.fused ? gp.splits : nb;
  // the bf16 split of the direction feeds only the separate JVP kernel
  const int split = gp.fused ? 0 : 1;

  HIPTRY(launch_tables(m, params, st));
  // mean energy, centred energies u = E_loc - E, variance partials
  hipLaunchKernelGGL((k_sum_e<C>), dim3(unsigned(nb)), dim3(256), 0, st, n,
                     (const double *)eloc, D(L.e_part));
  HIPTRY(hipGetLastError());
  hipLaunchKernelGGL((k_center_e<C>), dim3(unsigned(nb)), dim3(256), 0, st, n,
                     (const double *)eloc, D(L.e_part), nb, D(L.u), D(L.e_part2), state);
  HIPTRY(hipGetLastError());
  // chain means and their spread (error bar)
  const int64_t ncb = cdiv(nch, kChainsPerBlock), ncb2 = cdiv(nch, 256);
  hipLaunchKernelGGL((k_chain_mean<C>), dim3(unsigned(ncb)), dim3(256), 0, st, n, nch,
                     (const double *)eloc, D(L.cm), D(L.c_part));
  HIPTRY(hipGetLastError());
  hipLaunchKernelGGL(k_chain_dev, dim3(unsigned(ncb2)), dim3(256), 0, st, nch, D(L.cm),
                     D(L.c_part), ncb, D(L.c_part2));
  HIPTRY(hipGetLastError());
  // tanh(theta) of every sample, kept for all products of this step
  HIPTRY(launch_theta_tanh(m, sigma, n, grad, true, st));
  // O^dagger 1 (centring of S v), then g = O^dagger u (force numerator)
  hipLaunchKernelGGL((k_ones<C>), dim3(grid_for(n)), dim3(256), 0, st, n, D(L.y));
  HIPTRY(hipGetLastError());
  HIPTRY(launch_vjp_partials(m, sigma, n, D(L.y), grad, nullptr, st));
  HIPTRY(launch_vjp_reduce(m, n, grad, D(L.o1), nullptr, st));
  HIPTRY(launch_vjp_partials(m, sigma, n, D(L.u), grad, nullptr, st));
  HIPTRY(launch_vjp_reduce(m, n, grad, D(L.g), nullptr, st));
  hipLaunchKernelGGL((k_cg_init<T, C>), dim3(unsigned(pblocks)), dim3(256), 0, st, N, M, n,
                     D(L.e_part2), nb, D(L.g), D(L.F), D(L.x), D(L.r), D(L.p), (T *)gb.Vt,
                     (T *)gb.vb, gb.va, D(L.dpart), state, split);
  HIPTRY(hipGetLastError());
  hipLaunchKernelGGL(k_cg_start, dim3(1), dim3(256), 0, st, D(L.dpart), pblocks, cg_tol,
                     cg_maxiter, state, D(L.c_part2), ncb2, nch);
  HIPTRY(hipGetLastError());

  // Chunks of check_every iterations. The state after each chunk is copied to pinned host
  // memory behind the chunk, and the next chunk is queued before the host reads the copy,
  // so the device does not wait for the check; a chunk queued after convergence returns
  // at once in every kernel (the done flag).
  CGState *hslot = nullptr;
  CGState hs;
  const int check_every = 8;
  int launched = 0, queued = 0, checked = 0;
  const int *skip = &state->done;
  auto enqueue = [&](int batch, bool copy_back) -> nqs_status {
    // one CG iteration = the product's partial tiles, k_cg_apr, k_cg_xr, k_cg_p
    const int64_t ablocks = apr_blocks(elems, gp.splits);
    auto iterations = [&](int count, hipStream_t s2) -> hipError_t {
      for (int q = 0; q < count; ++q) {
        const int parity = q & 1;  // chunks start at an even iteration
        hipError_t e2;
        if (gp.fused) {
          e2 = launch_sv(m, sigma, n, grad, D(L.ysum), skip, s2, false);
        } else {
          e2 = launch_jvp(m, sigma, n, grad, D(L.y), D(L.ysum), skip, s2);
          if (e2 == hipSuccess)
            e2 = launch_vjp_partials(m, sigma, n, D(L.y), grad, skip, s2, false);
        }
        if (e2 != hipSuccess) return e2;
        k_cg_apr_launch<T, C>(elems, s2, N, M, n, gp.splits, gp.Itiles * 16,
                              (const T *)gb.part, D(L.o1), D(L.ysum), nys, D(L.p), diag_shift,
                              D(L.Ap), D(L.dpart), state);
        if ((e2 = hipGetLastError()) != hipSuccess) return e2;
        if (P <= kXrpMaxParams) {
          hipLaunchKernelGGL((k_cg_xrp<T, C>), dim3(1), dim3(kXrpThreads), 0, s2, N, M,
                             D(L.dpart), ablocks, parity, cg_tol, cg_maxiter, D(L.x), D(L.r),
                             D(L.p), D(L.Ap), (T *)gb.Vt, (T *)gb.vb, gb.va, state, split);
          if ((e2 = hipGetLastError()) != hipSuccess) return e2;
          continue;
        }
        hipLaunchKernelGGL(k_psum, dim3(1), dim3(1024), 0, s2, D(L.dpart), ablocks, D(L.psum),
                           (const CGState *)state);
        hipLaunchKernelGGL(k_cg_xr, dim3(unsigned(cblocks)), dim3(256), 0, s2, Pc, D(L.psum),
                           int64_t(1), parity, D(L.x), D(L.r), D(L.p), D(L.Ap), D(L.rpart), state);
        if ((e2 = hipGetLastError()) != hipSuccess) return e2;
        hipLaunchKernelGGL(k_psum, dim3(1), dim3(1024), 0, s2, D(L.rpart), cblocks, D(L.psum) + 1,
                           (const CGState *)state);
        hipLaunchKernelGGL((k_cg_p<T, C>), dim3(unsigned(pblocks)), dim3(256), 0, s2, N, M,
                           D(L.psum) + 1, int64_t(1), parity, cg_tol, cg_maxiter, D(L.r), D(L.p),
                           (T *)gb.Vt, (T *)gb.vb, gb.va, state, split);
        if ((e2 = hipGetLastError()) != hipSuccess) return e2;
      }
      return hipSuccess;
    };
    if (batch == check_every && m->cg_graphs) {
      // full chunks replay one captured graph: the arguments of the chunk's launches
      // depend only on the key below
      const CgGraphKey key{ws, sigma, n, diag_shift, cg_tol, cg_maxiter, m->sv_pairs};
      if (!m->cg_exec || !(m->cg_key == key)) {
        if (m->cg_exec) {
          (void)hipGraphExecDestroy(m->cg_exec);
          m->cg_exec = nullptr;
        }
        if (!m->cap_stream) HIPTRY(hipStreamCreate(&m->cap_stream));
        hipGraph_t graph = nullptr;
        HIPTRY(hipStreamBeginCapture(m->cap_stream, hipStreamCaptureModeThreadLocal));
        const hipError_t e1 = iterations(check_every, m->cap_stream);
        const hipError_t e2 = hipStreamEndCapture(m->cap_stream, &graph);
        if (e1 != hipSuccess || e2 != hipSuccess) {
          if (graph) (void)hipGraphDestroy(graph);
          return NQS_EDEVICE;
        }
        const hipError_t e3 = hipGraphInstantiate(&m->cg_exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e3 != hipSuccess) {
          m->cg_exec = nullptr;
          return NQS_EDEVICE;
        }
        m->cg_key = key;
      }
      HIPTRY(hipGraphLaunch(m->cg_exec, st));
    } else {
      HIPTRY(iterations(batch, st));
    }
    if (!copy_back) return NQS_OK;
    const int slot = queued & 1;
    HIPTRY(hipMemcpyAsync(&hslot[slot], state, sizeof(CGState), hipMemcpyDeviceToHost, st));
    HIPTRY(hipEventRecord(m->cg_ev[slot], st));
    ++queued;
    return NQS_OK;
  };
  auto launch_update = [&]() -> hipError_t {
    if (use_double(m))
      hipLaunchKernelGGL(k_update<double>, dim3(grid_for(Pc)), dim3(256), 0, st, Pc,
                         (double *)params, (const double *)D(L.x), lr, (const CGState *)state);
    else
      hipLaunchKernelGGL(k_update<float>, dim3(grid_for(Pc)), dim3(256), 0, st, Pc,
                         (float *)params, (const double *)D(L.x), lr, (const CGState *)state);
    return hipGetLastError();
  };
  if (async) {
    // every iteration slot is queued; the slots after the solve has finished return at
    // once. Chunks replay the cached graph unless the caller is capturing the stream (the
    // slots are then recorded into the caller's graph as plain launches).
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIPTRY(hipStreamIsCapturing(st, &cap));
    const bool saved = m->cg_graphs;
    if (cap != hipStreamCaptureStatusNone) m->cg_graphs = false;
    nqs_status qs = NQS_OK;
    for (int it = 0; it < cg_maxiter && qs == NQS_OK; it += check_every) {
      const int batch = cg_maxiter - it < check_every ? cg_maxiter - it : check_every;
      qs = enqueue(batch, false);
    }
    m->cg_graphs = saved;
    if (qs != NQS_OK) return qs;
    HIPTRY(launch_update());
    hipLaunchKernelGGL(k_sr_info, dim3(1), dim3(64), 0, st, (const CGState *)state, info);
    HIPTRY(hipGetLastError());
    return NQS_OK;
  }
  if (!m->cg_host) HIPTRY(hipHostMalloc(&m->cg_host, 2 * sizeof(CGState), hipHostMallocDefault));
  for (hipEvent_t &e : m->cg_ev)
    if (!e) HIPTRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  hslot = (CGState *)m->cg_host;
  // the state before the first chunk (k_cg_start may already have finished the solve)
  HIPTRY(hipMemcpyAsync(&hs, state, sizeof(CGState), hipMemcpyDeviceToHost, st));
  HIPTRY(hipStreamSynchronize(st));
  bool done = hs.done != 0;
  while (!done) {
    while (queued - checked < 2 && launched < cg_maxiter) {
      const int batch = cg_maxiter - launched < check_every ? cg_maxiter - launched : check_every;
      const nqs_status qs = enqueue(batch, true);
      if (qs != NQS_OK) return qs;
      launched += batch;
    }
    if (queued == checked) break;
    const int slot = checked & 1;
    HIPTRY(hipEventSynchronize(m->cg_ev[slot]));
    hs = hslot[slot];
    ++checked;
    done = hs.done != 0;
  }
  // chunks still queued return at once; the state no longer changes once done is set
  // (and the stream orders them before the update below)
  nqs_sr_info out;
  fill_info(hs, &out);
  if (out.status != NQS_ENONFINITE) HIPTRY(launch_update());
  HIPTRY(hipStreamSynchronize(st));
  if (info) *info = out;
  return nqs_status(out.status);
}

// SR step of a symmetric RBM (Sec. 2.2.2, 2.2.5): the samples' tanh(theta) rows and the
// Jacobian products of the expanded RBM, with the CG in the symmetric parameters:
// S_sym v = E^T S_exp E v, F_sym = E^T F_exp. Convergence is checked on the host after
// every chunk of 8 iterations (async: cg_maxiter slots, nothing read back).
template <typename T, bool C>
nqs_status sr_symm_impl(nqs_model *m, void *params, const int8_t *sigma, const void *eloc,
                        int64_t n, int64_t nch, double lr, double diag_shift, double cg_tol,
                        int cg_maxiter, void *ws, nqs_sr_info *info, bool async, hipStream_t st) {
  SRLayout L = sr_layout(m, n);
  char *b = (char *)ws;
  auto D = [&](size_t off) { return (double *)(b + off); };
  CGState *state = (CGState *)(b + L.state);
  void *grad = b + L.grad;
  const int cs = C ? 2 : 1;
  const int N = m->N, M = m->M;
  const int64_t Ps = n_params_model(m), Pcs = Ps * cs;
  const int64_t nb = cdiv(n, 256);
  const int64_t sblocks = cdiv(Ps, 256) < 4096 ? cdiv(Ps, 256) : 4096;
  const int64_t scblocks = cdiv(Pcs, 256) < 4096 ? cdiv(Pcs, 256) : 4096;
  const GradPlan gp = grad_plan(m, n);
  const GradBuffers gb = grad_buffers(m, n, grad);
  const int64_t elems = int64_t(gp.Jtiles) * 16 * gp.Itiles * 16;
  const int64_t nys = gp.fused ? gp.splits : nb;
  const int64_t ablocks = apr_blocks(elems, gp.splits);

  hipError_t e0;
  const void *pe = model_params(m, params, st, &e0);
  HIPTRY(e0);
  HIPTRY(launch_tables(m, pe, st));
  hipLaunchKernelGGL((k_sum_e<C>), dim3(unsigned(nb)), dim3(256), 0, st, n,
                     (const double *)eloc, D(L.e_part));
  HIPTRY(hipGetLastError());
  hipLaunchKernelGGL((k_center_e<C>), dim3(unsigned(nb)), dim3(256), 0, st, n,
                     (const double *)eloc, D(L.e_part), nb, D(L.u), D(L.e_part2), state);
  HIPTRY(hipGetLastError());
  const int64_t ncb = cdiv(nch, kChainsPerBlock), ncb2 = cdiv(nch, 256);
  hipLaunchKernelGGL((k_chain_mean<C>), dim3(unsigned(ncb)), dim3(256), 0, st, n, nch,
                     (const double *)eloc, D(L.cm), D(L.c_part));
  HIPTRY(hipGetLastError());
  hipLaunchKernelGGL(k_chain_dev, dim3(unsigned(ncb2)), dim3(256), 0, st, nch, D(L.cm),
                     D(L.c_part), ncb, D(L.c_part2));
  HIPTRY(hipGetLastError());
  HIPTRY(launch_theta_tanh(m, sigma, n, grad, true, st));
  // O^dagger 1 and the force numerator, expanded, then summed to the symmetric parameters
  hipLaunchKernelGGL((k_ones<C>), dim3(grid_for(n)), dim3(256), 0, st, n, D(L.y));
  HIPTRY(hipGetLastError());
  HIPTRY(launch_vjp_partials(m, sigma, n, D(L.y), grad, nullptr, st));
  HIPTRY(launch_vjp_reduce(m, n, grad, D(L.o1), nullptr, st));
  HIPTRY(launch_symm_reduce(m, D(L.o1), D(L.o1s), st));
  HIPTRY(launch_vjp_partials(m, sigma, n, D(L.u), grad, nullptr, st));
  HIPTRY(launch_vjp_reduce(m, n, grad, D(L.g), nullptr, st));
  HIPTRY(launch_symm_reduce(m, D(L.g), D(L.gs), st));
  (void)M;
  hipLaunchKernelGGL((k_symm_cg_init<C>), dim3(unsigned(sblocks)), dim3(256), 0, st, Ps, n,
                     D(L.e_part2), nb, D(L.gs), D(L.F), D(L.x), D(L.r), D(L.p), D(L.dpart),
                     state);
  HIPTRY(hipGetLastError());
  hipLaunchKernelGGL(k_cg_start, dim3(1), dim3(256), 0, st, D(L.dpart), sblocks, cg_tol,
                     cg_maxiter, state, D(L.c_part2), ncb2, nch);
  HIPTRY(hipGetLastError());
  const int *skip = &state->done;
  auto iteration = [&](int parity) -> hipError_t {
    hipError_t e = launch_symm_expand_dir(m, D(L.p), D(L.vexp), skip, st);
    if (e == hipSuccess) e = launch_prep_dir(m, D(L.vexp), grad, !gp.fused, st);
    if (e != hipSuccess) return e;
    if (gp.fused) {
      e = launch_sv(m, sigma, n, grad, D(L.ysum), skip, st, false);
    } else {
      e = launch_jvp(m, sigma, n, grad, D(L.y), D(L.ysum), skip, st);
      if (e == hipSuccess) e = launch_vjp_partials(m, sigma, n, D(L.y), grad, skip, st, false);
    }
    if (e != hipSuccess) return e;
    // expanded (g - ybar O^dagger 1) / n, then summed over the symmetry copies
    k_cg_apr_launch<T, C>(elems, st, N, m->M, n, gp.splits, gp.Itiles * 16, (const T *)gb.part,
                          D(L.o1), D(L.ysum), nys, D(L.vexp), 0.0, D(L.apexp), D(L.dpart), state);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_symm_reduce(m, D(L.apexp), D(L.Ap), st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_symm_shift_dot, dim3(unsigned(sblocks)), dim3(256), 0, st, Pcs,
                       D(L.p), diag_shift, D(L.Ap), D(L.dpart), (const CGState *)state);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_psum, dim3(1), dim3(1024), 0, st, D(L.dpart), sblocks, D(L.psum),
                       (const CGState *)state);
    hipLaunchKernelGGL(k_cg_xr, dim3(unsigned(scblocks)), dim3(256), 0, st, Pcs, D(L.psum),
                       int64_t(1), parity, D(L.x), D(L.r), D(L.p), D(L.Ap), D(L.rpart), state);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_psum, dim3(1), dim3(1024), 0, st, D(L.rpart), scblocks, D(L.psum) + 1,
                       (const CGState *)state);
    hipLaunchKernelGGL(k_cg_p_plain, dim3(unsigned(scblocks)), dim3(256), 0, st, Pcs,
                       D(L.psum) + 1, int64_t(1), parity, cg_tol, cg_maxiter, D(L.r), D(L.p),
                       state);
    return hipGetLastError();
  };
  auto update = [&]() -> hipError_t {
    if (use_double(m))
      hipLaunchKernelGGL(k_update<double>, dim3(grid_for(Pcs)), dim3(256), 0, st, Pcs,
                         (double *)params, (const double *)D(L.x), lr, (const CGState *)state);
    else
      hipLaunchKernelGGL(k_update<float>, dim3(grid_for(Pcs)), dim3(256), 0, st, Pcs,
                         (float *)params, (const double *)D(L.x), lr, (const CGState *)state);
    return hipGetLastError();
  };
  if (async) {
    for (int it = 0; it < cg_maxiter; ++it) HIPTRY(iteration(it & 1));
    HIPTRY(update());
    hipLaunchKernelGGL(k_sr_info, dim3(1), dim3(64), 0, st, (const CGState *)state, info);
    HIPTRY(hipGetLastError());
    return NQS_OK;
  }
  CGState hs;
  int launched = 0;
  for (;;) {
    HIPTRY(hipMemcpyAsync(&hs, state, sizeof(CGState), hipMemcpyDeviceToHost, st));
    HIPTRY(hipStreamSynchronize(st));
    if (hs.done || launched >= cg_maxiter) break;
    const int batch = cg_maxiter - launched < 8 ? cg_maxiter - launched : 8;
    for (int q = 0; q < batch; ++q, ++launched) HIPTRY(iteration(launched & 1));
  }
  nqs_sr_info out;
  fill_info(hs, &out);
  if (out.status != NQS_ENONFINITE) HIPTRY(update());
  HIPTRY(hipStreamSynchronize(st));
  if (info) *info = out;
  return nqs_status(out.status);
}

// ---- feed-forward network: the same CG with the network's Jacobian products ----------
// ybar = mean of y = O p from the JVP's block partials (fixed order)
__global__ __launch_bounds__(256) void k_ff_ybar(const double *ysum, int64_t nparts, int64_t n,
                                                 double *ybar, const CGState *st) {
  if (st && st->done) return;
  __shared__ double lds[256];
  const double a = block_sum(ysum, nparts, 2, lds);
  const double b = block_sum(ysum + 1, nparts, 2, lds);
  if (threadIdx.x == 0) {
    ybar[0] = a / double(n);
    ybar[1] = b / double(n);
  }
}

// Ap = (O^dagger y - ybar O^dagger 1) / n, in place on O^dagger y
template <bool C>
__global__ void k_ff_apr(int64_t P, int64_t n, const double *o1, const double *ybar,
                         double *Ap, const CGState *st) {
  if (st && st->done) return;
  const double yr = ybar[0], yi = C ? ybar[1] : 0.0, inv = 1.0 / double(n);
  for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < P;
       k += int64_t(gridDim.x) * blockDim.x) {
    if (C) {
      const double orr = o1[2 * k], oi = o1[2 * k + 1];
      Ap[2 * k] = (Ap[2 * k] - (yr * orr - yi * oi)) * inv;
      Ap[2 * k + 1] = (Ap[2 * k + 1] - (yr * oi + yi * orr)) * inv;
    } else {
      Ap[k] = (Ap[k] - yr * o1[k]) * inv;
    }
  }
}

template <typename T, bool C>
nqs_status sr_ff_impl(nqs_model *m, void *params, const int8_t *sigma, const void *eloc,
                      int64_t n, int64_t nch, double lr, double diag_shift, double cg_tol,
                      int cg_maxiter, void *ws, nqs_sr_info *info, bool async, hipStream_t st) {
  SRLayout L = sr_layout(m, n);
  char *b = (char *)ws;
  auto D = [&](size_t off) { return (double *)(b + off); };
  CGState *state = (CGState *)(b + L.state);
  void *grad = b + L.grad;
  const int cs = C ? 2 : 1;
  const int64_t Ps = n_params_model(m), Pcs = Ps * cs;
  const int64_t nb = cdiv(n, 256);
  const int64_t sblocks = cdiv(Ps, 256) < 4096 ? cdiv(Ps, 256) : 4096;
  const int64_t scblocks = cdiv(Pcs, 256) < 4096 ? cdiv(Pcs, 256) : 4096;
  const int64_t jb = ff_jvp_blocks(m, n);

  HIPTRY(launch_ff_tables(m, params, st));
  hipLaunchKernelGGL((k_sum_e<C>), dim3(unsigned(nb)), dim3(256), 0, st, n,
                     (const double *)eloc, D(L.e_part));
  HIPTRY(hipGetLastError());
  hipLaunchKernelGGL((k_center_e<C>), dim3(unsigned(nb)), dim3(256), 0, st, n,
                     (const double *)eloc, D(L.e_part), nb, D(L.u), D(L.e_part2), state);
  HIPTRY(hipGetLastError());
  const int64_t ncb = cdiv(nch, kChainsPerBlock), ncb2 = cdiv(nch, 256);
  hipLaunchKernelGGL((k_chain_mean<C>), dim3(unsigned(ncb)), dim3(256), 0, st, n, nch,
                     (const double *)eloc, D(L.cm), D(L.c_part));
  HIPTRY(hipGetLastError());
  hipLaunchKernelGGL(k_chain_dev, dim3(unsigned(ncb2)), dim3(256), 0, st, nch, D(L.cm),
                     D(L.c_part), ncb, D(L.c_part2));
  HIPTRY(hipGetLastError());
  // the network's rows, O^dagger 1 and the force numerator
  HIPTRY(launch_ff_fb(m, params, sigma, n, grad, st));
  hipLaunchKernelGGL((k_ones<C>), dim3(grid_for(n)), dim3(256), 0, st, n, D(L.y));
  HIPTRY(hipGetLastError());
  HIPTRY(launch_ff_vjp(m, sigma, n, D(L.y), grad, D(L.o1), nullptr, st));
  HIPTRY(launch_ff_vjp(m, sigma, n, D(L.u), grad, D(L.g), nullptr, st));
  hipLaunchKernelGGL((k_symm_cg_init<C>), dim3(unsigned(sblocks)), dim3(256), 0, st, Ps, n,
                     D(L.e_part2), nb, D(L.g), D(L.F), D(L.x), D(L.r), D(L.p), D(L.dpart),
                     state);
  HIPTRY(hipGetLastError());
  hipLaunchKernelGGL(k_cg_start, dim3(1), dim3(256), 0, st, D(L.dpart), sblocks, cg_tol,
                     cg_maxiter, state, D(L.c_part2), ncb2, nch);
  HIPTRY(hipGetLastError());
  const int *skip = &state->done;
  auto iteration = [&](int parity) -> hipError_t {
    hipError_t e = launch_ff_jvp(m, params, sigma, n, D(L.p), grad, D(L.y), D(L.ysum), skip, st);
    if (e == hipSuccess) e = launch_ff_vjp(m, sigma, n, D(L.y), grad, D(L.Ap), skip, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ff_ybar, dim3(1), dim3(256), 0, st, D(L.ysum), jb, n, D(L.ybar),
                       (const CGState *)state);
    hipLaunchKernelGGL((k_ff_apr<C>), dim3(unsigned(sblocks)), dim3(256), 0, st, Ps, n,
                       D(L.o1), D(L.ybar), D(L.Ap), (const CGState *)state);
    hipLaunchKernelGGL(k_symm_shift_dot, dim3(unsigned(sblocks)), dim3(256), 0, st, Pcs,
                       D(L.p), diag_shift, D(L.Ap), D(L.dpart), (const CGState *)state);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_psum, dim3(1), dim3(1024), 0, st, D(L.dpart), sblocks, D(L.psum),
                       (const CGState *)state);
    hipLaunchKernelGGL(k_cg_xr, dim3(unsigned(scblocks)), dim3(256), 0, st, Pcs, D(L.psum),
                       int64_t(1), parity, D(L.x), D(L.r), D(L.p), D(L.Ap), D(L.rpart), state);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_psum, dim3(1), dim3(1024), 0, st, D(L.rpart), scblocks, D(L.psum) + 1,
                       (const CGState *)state);
    hipLaunchKernelGGL(k_cg_p_plain, dim3(unsigned(scblocks)), dim3(256), 0, st, Pcs,
                       D(L.psum) + 1, int64_t(1), parity, cg_tol, cg_maxiter, D(L.r), D(L.p),
                       state);
    return hipGetLastError();
  };
  auto update = [&]() -> hipError_t {
    hipLaunchKernelGGL(k_update<T>, dim3(grid_for(Pcs)), dim3(256), 0, st, Pcs, (T *)params,
                       (const double *)D(L.x), lr, (const CGState *)state);
    return hipGetLastError();
  };
  if (async) {
    for (int it = 0; it < cg_maxiter; ++it) HIPTRY(iteration(it & 1));
    HIPTRY(update());
    hipLaunchKernelGGL(k_sr_info, dim3(1), dim3(64), 0, st, (const CGState *)state, info);
    HIPTRY(hipGetLastError());
    return NQS_OK;
  }
  CGState hs;
  int launched = 0;
  for (;;) {
    HIPTRY(hipMemcpyAsync(&hs, state, sizeof(CGState), hipMemcpyDeviceToHost, st));
    HIPTRY(hipStreamSynchronize(st));
    if (hs.done || launched >= cg_maxiter) break;
    const int batch = cg_maxiter - launched < 8 ? cg_maxiter - launched : 8;
    for (int q = 0; q < batch; ++q, ++launched) HIPTRY(iteration(launched & 1));
  }
  nqs_sr_info out;
  fill_info(hs, &out);
  if (out.status != NQS_ENONFINITE) HIPTRY(update());
  HIPTRY(hipStreamSynchronize(st));
  if (info) *info = out;
  return nqs_status(out.status);
}

template <bool C>
nqs_status prepare_impl(nqs_model *m, const void *params, const int8_t *sigma, int64_t n,
                        void *ws, hipStream_t st) {
  SRLayout L = sr_layout(m, n);
  char *b = (char *)ws;
  void *grad = b + L.grad;
  hipError_t e0;
  params = model_params(m, params, st, &e0);
  HIPTRY(e0);
  HIPTRY(launch_tables(m, params, st));
  HIPTRY(launch_theta_tanh(m, sigma, n, grad, true, st));
  hipLaunchKernelGGL((k_ones<C>), dim3(grid_for(n)), dim3(256), 0, st, n, (double *)(b + L.y));
  HIPTRY(hipGetLastError());
  HIPTRY(launch_vjp_partials(m, sigma, n, (double *)(b + L.y), grad, nullptr, st));
  HIPTRY(launch_vjp_reduce(m, n, grad, (double *)(b + L.o1), nullptr, st));
  return NQS_OK;
}

template <bool C>
nqs_status matvec_impl(nqs_model *m, const int8_t *sigma, int64_t n, void *ws, const void *v,
                       double lambda, void *out, hipStream_t st) {
  SRLayout L = sr_layout(m, n);
  char *b = (char *)ws;
  void *grad = b + L.grad;
  const GradPlan gp = grad_plan(m, n);
  const GradBuffers gb = grad_buffers(m, n, grad);
  const int64_t elems = int64_t(gp.Jtiles) * 16 * gp.Itiles * 16;
  // symmetric RBM: the product of the expanded RBM on E v, summed back over the copies
  const void *v_in = v;
  void *out_sym = out;
  if (m->G) {
    HIPTRY(launch_symm_expand_dir(m, (const double *)v, (double *)(b + L.vexp), nullptr, st));
    v = b + L.vexp;
    out = b + L.apexp;
  }
  const double lambda_exp = m->G ? 0.0 : lambda;
  // (timing marks around each launcher: the product's kernel time without the gaps)
  time_begin(m, NQS_TIME_SV);
  time_mark(m, NQS_TIME_SV, 0, st);
  HIPTRY(launch_prep_dir(m, v, grad, !gp.fused, st));
  time_mark(m, NQS_TIME_SV, 1, st);
  // the partial tiles of the product, summed over the sample splits by the kernel of the
  // CG iterations (no solver state)
  time_mark(m, NQS_TIME_SV, 0, st);
  if (gp.fused) {
    HIPTRY(launch_sv(m, sigma, n, grad, (double *)(b + L.ysum), nullptr, st, false));
  } else {
    HIPTRY(launch_jvp(m, sigma, n, grad, (double *)(b + L.y), (double *)(b + L.ysum), nullptr, st));
    time_mark(m, NQS_TIME_SV, 1, st);
    time_mark(m, NQS_TIME_SV, 0, st);
    HIPTRY(launch_vjp_partials(m, sigma, n, (double *)(b + L.y), grad, nullptr, st, false));
  }
  time_mark(m, NQS_TIME_SV, 1, st);
  time_mark(m, NQS_TIME_SV, 0, st);
  const int64_t nys = gp.fused ? gp.splits : cdiv(n, 256);
  auto apr = [&](auto tc) {
    typedef decltype(tc) T;
    k_cg_apr_launch<T, C>(elems, st, m->N, m->M, n, gp.splits, gp.Itiles * 16,
                          (const T *)gb.part, (const double *)(b + L.o1),
                          (const double *)(b + L.ysum), nys, (const double *)v, lambda_exp,
                          (double *)out, (double *)(b + L.dpart), (const CGState *)nullptr);
  };
  if (use_double(m))
    apr(double(0));
  else
    apr(float(0));
  HIPTRY(hipGetLastError());
  if (m->G) {
    HIPTRY(launch_symm_reduce(m, (const double *)out, (double *)out_sym, st));
    const int64_t Pcs = n_params_model(m) * (C ? 2 : 1);
    hipLaunchKernelGGL(k_symm_shift_dot, dim3(grid_for(Pcs)), dim3(256), 0, st, Pcs,
                       (const double *)v_in, lambda, (double *)out_sym, (double *)nullptr,
                       (const CGState *)nullptr);
    HIPTRY(hipGetLastError());
  }
  time_mark(m, NQS_TIME_SV, 1, st);
  return NQS_OK;
}

// ---------------------------------------------------------------------------------
// Batched SR (nqs_batch): every model's solve advances in the same launches. Each block
// reads its model's job and its block index from a block map and runs the single-model
// body; models whose CG has finished return at once (their state's done flag).
// ---------------------------------------------------------------------------------
template <typename T>
struct BJob {
  int N, M;
  int64_t n, P, Pc, nb;
  int64_t nch, ncb, ncb2;  // chains of the error bar, blocks of the chain-mean kernels
  double *cm, *cpart, *cpart2;
  int pblocks, cblocks, colsP;
  int64_t elems;
  const double *e;
  double *epart, *epart2, *u, *ones;
  double *g, *F, *x, *r, *p, *Ap, *o1, *dpart, *rpart;
  const double *out1, *ysum;
  T *Vt, *vb;
  double *va;
  void *params;
  CGState *st;
};

// the solver states of all models of a batch, gathered for one host read
template <typename T>
__global__ void kb_gather_states(const BJob<T> *jobs, int K, CGState *out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < K) out[k] = *jobs[k].st;
}

template <typename T, bool C>
__global__ __launch_bounds__(256) void kb_stats1(const BJob<T> *jobs, const int2 *map) {
  const int2 b = map[blockIdx.x];
  const BJob<T> J = jobs[b.x];
  k_sum_e_body<C>(b.y, 0, 0, 0, J.n, J.e, J.epart);
}
template <typename T, bool C>
__global__ __launch_bounds__(256) void kb_stats2(const BJob<T> *jobs, const int2 *map) {
  const int2 b = map[blockIdx.x];
  const BJob<T> J = jobs[b.x];
  k_center_e_body<C>(b.y, 0, 0, 0, J.n, J.e, J.epart, J.nb, J.u, J.epart2, J.st);
  // O^dagger 1 needs a vector of ones
  const int64_t s = int64_t(b.y) * 256 + threadIdx.x;
  if (s < J.n) {
    if (C) {
      J.ones[2 * s] = 1.0;
      J.ones[2 * s + 1] = 0.0;
    } else {
      J.ones[s] = 1.0;
    }
  }
}
template <typename T, bool C>
__global__ __launch_bounds__(256) void kb_chain_mean(const BJob<T> *jobs, const int2 *map) {
  const int2 b = map[blockIdx.x];
  const BJob<T> J = jobs[b.x];
  k_chain_mean_body<C>(b.y, J.n, J.nch, J.e, J.cm, J.cpart);
}
template <typename T>
__global__ __launch_bounds__(256) void kb_chain_dev(const BJob<T> *jobs, const int2 *map) {
  const int2 b = map[blockIdx.x];
  const BJob<T> J = jobs[b.x];
  k_chain_dev_body(b.y, J.nch, J.cm, J.cpart, J.ncb, J.cpart2);
}
template <typename T>
__global__ void kb_info(const BJob<T> *jobs, int K, nqs_sr_info *out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < K) fill_info(*jobs[k].st, out + k);
}
template <typename T, bool C>
__global__ __launch_bounds__(256) void kb_cg_init(const BJob<T> *jobs, const int2 *map) {
  const int2 b = map[blockIdx.x];
  const BJob<T> J = jobs[b.x];
  k_cg_init_body<T, C>(b.y, 0, 0, J.pblocks, J.N, J.M, J.n, J.epart2, J.nb, J.g, J.F, J.x, J.r,
                       J.p, J.Vt, J.vb, J.va, J.dpart, J.st, 1);
}
template <typename T>
__global__ __launch_bounds__(256) void kb_cg_start(const BJob<T> *jobs, double tol,
                                                   int maxiter) {
  const BJob<T> J = jobs[blockIdx.x];
  k_cg_start_body(0, 0, 0, 1, J.dpart, J.pblocks, tol, maxiter, J.st, J.cpart2, J.ncb2, J.nch);
}
template <typename T, bool C>
__global__ __launch_bounds__(256) void kb_cg_ap(const BJob<T> *jobs, const int2 *map,
                                                double lambda) {
  const int2 b = map[blockIdx.x];
  const BJob<T> J = jobs[b.x];
  k_cg_ap_body<C>(b.y, 0, 0, J.pblocks, J.N, J.M, J.n, 1, J.colsP, J.elems, J.out1, J.o1,
                  J.ysum, J.nb, J.p, lambda, J.Ap, J.dpart, J.st);
}
template <typename T>
__global__ __launch_bounds__(256) void kb_cg_xr(const BJob<T> *jobs, const int2 *map,
                                                int parity) {
  const int2 b = map[blockIdx.x];
  const BJob<T> J = jobs[b.x];
  k_cg_xr_body(b.y, 0, 0, J.cblocks, J.Pc, J.dpart, J.pblocks, parity, J.x, J.r, J.p, J.Ap,
               J.rpart, J.st);
}
template <typename T, bool C>
__global__ __launch_bounds__(256) void kb_cg_p(const BJob<T> *jobs, const int2 *map,
                                               int parity, double tol, int maxiter) {
  const int2 b = map[blockIdx.x];
  const BJob<T> J = jobs[b.x];
  k_cg_p_body<T, C>(b.y, 0, 0, J.pblocks, J.N, J.M, J.rpart, J.cblocks, parity, tol, maxiter,
                    J.r, J.p, J.Vt, J.vb, J.va, J.st, 1);
}
// parameter update of the models whose energy and solve are finite
template <typename T, typename PT>
__global__ __launch_bounds__(256) void kb_update(const BJob<T> *jobs, const int2 *map,
                                                 double lr) {
  const int2 b = map[blockIdx.x];
  const BJob<T> J = jobs[b.x];
  if (!step_finite(J.st)) return;
  k_update_body<PT>(b.y, 0, 0, J.cblocks, J.Pc, (PT *)J.params, J.x, lr);
}

struct BLayout {
  size_t Tm, Vt, vb, va, ypart, part, out1, y, ysum, u, ones, epart, epart2, cm, cpart, cpart2,
      o1, g, F, x, r, p, Ap, dpart, rpart, state, total;
};

BLayout batch_layout(const nqs_model *m, int64_t n) {
  const int cs = m->is_complex ? 2 : 1;
  const int64_t P = int64_t(m->N) + m->M + int64_t(m->N) * m->M;
  const int64_t nb = cdiv(n, 256);
  const int64_t pb = cdiv(P, 256) < 4096 ? cdiv(P, 256) : 4096;
  const int64_t cb = cdiv(P * cs, 256) < 4096 ? cdiv(P * cs, 256) : 4096;
  const BatchGradSizes z = batch_grad_sizes(m, n);
  BLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += (bytes + 255) / 256 * 256;
    return o;
  };
  L.Tm = take(z.Tm);
  L.Vt = take(z.Vt);
  L.vb = take(z.vb);
  L.va = take(z.va);
  L.ypart = take(z.ypart);
  L.part = take(z.part);
  L.out1 = take(z.out1);
  L.y = take(size_t(n) * cs * 8);
  L.ysum = take(size_t(nb) * 16);
  L.u = take(size_t(n) * cs * 8);
  L.ones = take(size_t(n) * cs * 8);
  L.epart = take(size_t(nb) * 16);
  L.epart2 = take(size_t(nb) * 8);
  L.cm = take(size_t(n) * 8);
  L.cpart = take(size_t(cdiv(n, kChainsPerBlock)) * 8);
  L.cpart2 = take(size_t(nb) * 8);
  L.o1 = take(size_t(P) * cs * 8);
  L.g = take(size_t(P) * cs * 8);
  L.F = take(size_t(P) * cs * 8);
  L.x = take(size_t(P) * cs * 8);
  L.r = take(size_t(P) * cs * 8);
  L.p = take(size_t(P) * cs * 8);
  L.Ap = take(size_t(P) * cs * 8);
  L.dpart = take(size_t(pb) * 8);
  L.rpart = take(size_t(cb) * 8);
  L.state = take(sizeof(CGState));
  L.total = off;
  return L;
}

// job-table slots of the batch handle used by the SR step
enum { kSlotJobs = 0, kSlotStats, kSlotP, kSlotC, kSlotStart, kSlotChains = 5, kSlotStates = 6,
       kSlotChainDev = 7, kSlotTanh = 10,
       kSlotJvp = 12,
       kSlotVjp1 = 16, kSlotVjpU = 20, kSlotVjpY = 24 };

template <typename T, bool C>
nqs_status batch_sr_impl(nqs_batch *b, void *params, const int8_t *samples, const void *eloc,
                         const int64_t *n_samples, const int32_t *n_chains, double lr,
                         double diag_shift, double cg_tol, int cg_maxiter, void *ws,
                         nqs_sr_info *info, bool async, hipStream_t st) {
  typedef typename std::conditional<std::is_same<T, double>::value, double, float>::type PT;
  const int K = b->K;
  const int cs = C ? 2 : 1;
  std::vector<BJob<T>> jobs(K);
  std::vector<BatchGradItem> gi(K);
  std::vector<const void *> pk(K);
  std::vector<int2> map_s, map_p, map_c, map_m, map_d;
  std::vector<CGState *> states(K);
  size_t wo = 0, po = 0, so = 0, eo = 0;
  for (int k = 0; k < K; ++k) {
    const nqs_model *m = b->models[k];
    const int64_t n = n_samples[k];
    const BLayout L = batch_layout(m, n);
    char *w = (char *)ws + wo;
    const int64_t P = int64_t(m->N) + m->M + int64_t(m->N) * m->M;
    BJob<T> &J = jobs[k];
    memset(static_cast<void *>(&J), 0, sizeof(J));  // compared byte by byte with the last upload
    J.N = m->N;
    J.M = m->M;
    J.n = n;
    J.P = P;
    J.Pc = P * cs;
    J.nb = cdiv(n, 256);
    J.pblocks = int(cdiv(P, 256) < 4096 ? cdiv(P, 256) : 4096);
    J.cblocks = int(cdiv(P * cs, 256) < 4096 ? cdiv(P * cs, 256) : 4096);
    J.nch = (n_chains && n_chains[k] > 0) ? n_chains[k] : n;
    J.ncb = cdiv(J.nch, kChainsPerBlock);
    J.ncb2 = cdiv(J.nch, 256);
    J.cm = (double *)(w + L.cm);
    J.cpart = (double *)(w + L.cpart);
    J.cpart2 = (double *)(w + L.cpart2);
    const BatchGradSizes z = batch_grad_sizes(m, n);
    J.colsP = z.colsP;
    J.elems = z.elems;
    J.e = (const double *)((const char *)eloc + eo);
    J.epart = (double *)(w + L.epart);
    J.epart2 = (double *)(w + L.epart2);
    J.u = (double *)(w + L.u);
    J.ones = (double *)(w + L.ones);
    J.g = (double *)(w + L.g);
    J.F = (double *)(w + L.F);
    J.x = (double *)(w + L.x);
    J.r = (double *)(w + L.r);
    J.p = (double *)(w + L.p);
    J.Ap = (double *)(w + L.Ap);
    J.o1 = (double *)(w + L.o1);
    J.dpart = (double *)(w + L.dpart);
    J.rpart = (double *)(w + L.rpart);
    J.out1 = (const double *)(w + L.out1);
    J.ysum = (const double *)(w + L.ysum);
    J.Vt = (T *)(w + L.Vt);
    J.vb = (T *)(w + L.vb);
    J.va = (double *)(w + L.va);
    J.params = (char *)params + po;
    J.st = (CGState *)(w + L.state);
    states[k] = J.st;
    pk[k] = J.params;
    BatchGradItem &G = gi[k];
    G.m = m;
    G.n = n;
    G.sigma = samples + so;
    G.Tm = w + L.Tm;
    G.Vt = w + L.Vt;
    G.vb = w + L.vb;
    G.va = (double *)(w + L.va);
    G.ypart = (double *)(w + L.ypart);
    G.y = (double *)(w + L.y);
    G.ysum = (double *)(w + L.ysum);
    G.u = nullptr;
    G.part = w + L.part;
    G.out1 = (double *)(w + L.out1);
    G.out = nullptr;
    G.skip = nullptr;
    for (int x = 0; x < int(J.nb); ++x) map_s.push_back(make_int2(k, x));
    for (int x = 0; x < J.pblocks; ++x) map_p.push_back(make_int2(k, x));
    for (int x = 0; x < J.cblocks; ++x) map_c.push_back(make_int2(k, x));
    for (int x = 0; x < int(J.ncb); ++x) map_m.push_back(make_int2(k, x));
    for (int x = 0; x < int(J.ncb2); ++x) map_d.push_back(make_int2(k, x));
    wo += L.total;
    po += size_t(P) * cs * (std::is_same<T, double>::value ? 8 : 4);
    so += size_t(n) * m->N;
    eo += size_t(n) * cs * 8;
  }
  hipError_t e;
#define BTRY(x)                            \
  do {                                     \
    if ((e = (x)) != hipSuccess) return NQS_EDEVICE; \
  } while (0)
  BTRY(b->buf(kSlotJobs).upload(jobs.data(), jobs.size() * sizeof(BJob<T>), st));
  BTRY(b->buf(kSlotStats).upload(map_s.data(), map_s.size() * sizeof(int2), st));
  BTRY(b->buf(kSlotP).upload(map_p.data(), map_p.size() * sizeof(int2), st));
  BTRY(b->buf(kSlotC).upload(map_c.data(), map_c.size() * sizeof(int2), st));
  BTRY(b->buf(kSlotChains).upload(map_m.data(), map_m.size() * sizeof(int2), st));
  BTRY(b->buf(kSlotChainDev).upload(map_d.data(), map_d.size() * sizeof(int2), st));
  if (!b->buf(kSlotJobs).d || !b->buf(kSlotStats).d || !b->buf(kSlotP).d || !b->buf(kSlotC).d ||
      !b->buf(kSlotChains).d || !b->buf(kSlotChainDev).d)
    return NQS_EDEVICE;
  const BJob<T> *dj = (const BJob<T> *)b->buf(kSlotJobs).d;
  const int2 *ms = (const int2 *)b->buf(kSlotStats).d;
  const int2 *mp = (const int2 *)b->buf(kSlotP).d;
  const int2 *mc = (const int2 *)b->buf(kSlotC).d;

  BTRY(launch_tables_batch(b, pk, st));
  hipLaunchKernelGGL((kb_stats1<T, C>), dim3(unsigned(map_s.size())), dim3(256), 0, st, dj, ms);
  BTRY(hipGetLastError());
  hipLaunchKernelGGL((kb_stats2<T, C>), dim3(unsigned(map_s.size())), dim3(256), 0, st, dj, ms);
  BTRY(hipGetLastError());
  hipLaunchKernelGGL((kb_chain_mean<T, C>), dim3(unsigned(map_m.size())), dim3(256), 0, st, dj,
                     (const int2 *)b->buf(kSlotChains).d);
  BTRY(hipGetLastError());
  hipLaunchKernelGGL((kb_chain_dev<T>), dim3(unsigned(map_d.size())), dim3(256), 0, st, dj,
                     (const int2 *)b->buf(kSlotChainDev).d);
  BTRY(hipGetLastError());
  BTRY(launch_theta_tanh_batch(b, gi, kSlotTanh, st));
  // O^dagger 1 and the force numerator g = O^dagger (E - E)
  for (int k = 0; k < K; ++k) {
    gi[k].u = jobs[k].ones;
    gi[k].out = jobs[k].o1;
  }
  BTRY(launch_vjp_batch(b, gi, true, kSlotVjp1, st));
  for (int k = 0; k < K; ++k) {
    gi[k].u = jobs[k].u;
    gi[k].out = jobs[k].g;
  }
  BTRY(launch_vjp_batch(b, gi, true, kSlotVjpU, st));
  hipLaunchKernelGGL((kb_cg_init<T, C>), dim3(unsigned(map_p.size())), dim3(256), 0, st, dj, mp);
  BTRY(hipGetLastError());
  hipLaunchKernelGGL((kb_cg_start<T>), dim3(unsigned(K)), dim3(256), 0, st, dj, cg_tol,
                     cg_maxiter);
  BTRY(hipGetLastError());
  // CG products: y = O p, then O^dagger y into the tile sums read by kb_cg_ap
  for (int k = 0; k < K; ++k) {
    gi[k].u = gi[k].y;
    gi[k].out = nullptr;
    gi[k].skip = &states[k]->done;
  }
  auto iteration = [&](int parity) -> hipError_t {
    hipError_t e2 = launch_jvp_batch(b, gi, kSlotJvp, st);
    if (e2 == hipSuccess) e2 = launch_vjp_batch(b, gi, false, kSlotVjpY, st);
    if (e2 != hipSuccess) return e2;
    hipLaunchKernelGGL((kb_cg_ap<T, C>), dim3(unsigned(map_p.size())), dim3(256), 0, st, dj, mp,
                       diag_shift);
    if ((e2 = hipGetLastError()) != hipSuccess) return e2;
    hipLaunchKernelGGL((kb_cg_xr<T>), dim3(unsigned(map_c.size())), dim3(256), 0, st, dj, mc,
                       parity);
    if ((e2 = hipGetLastError()) != hipSuccess) return e2;
    hipLaunchKernelGGL((kb_cg_p<T, C>), dim3(unsigned(map_p.size())), dim3(256), 0, st, dj, mp,
                       parity, cg_tol, cg_maxiter);
    return hipGetLastError();
  };
  if (async) {
    // every iteration slot is queued; finished models return at once in every kernel
    for (int it = 0; it < cg_maxiter; ++it) BTRY(iteration(it & 1));
    hipLaunchKernelGGL((kb_update<T, PT>), dim3(unsigned(map_c.size())), dim3(256), 0, st, dj,
                       mc, lr);
    BTRY(hipGetLastError());
    hipLaunchKernelGGL((kb_info<T>), dim3(unsigned((K + 63) / 64)), dim3(64), 0, st, dj, K, info);
    BTRY(hipGetLastError());
    return NQS_OK;
  }
  std::vector<CGState> hs(K);
  // every model's solver state is gathered into one device array and read in one copy
  BTRY(b->buf(kSlotStates).upload(hs.data(), hs.size() * sizeof(CGState), st));
  if (!b->buf(kSlotStates).d) return NQS_EDEVICE;
  CGState *dstates = (CGState *)b->buf(kSlotStates).d;
  // chunks of check_every iterations; the gathered states after each chunk are copied to
  // pinned host memory behind it, and the next chunk is queued before the host reads them
  const size_t hbytes = 2 * size_t(K) * sizeof(CGState);
  if (b->cg_host_bytes < hbytes) {
    if (b->cg_host) BTRY(hipHostFree(b->cg_host));
    b->cg_host = nullptr;
    b->cg_host_bytes = 0;
    BTRY(hipHostMalloc(&b->cg_host, hbytes, hipHostMallocDefault));
    b->cg_host_bytes = hbytes;
  }
  for (hipEvent_t &ev : b->cg_ev)
    if (!ev) BTRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  CGState *hslot = (CGState *)b->cg_host;
  const int check_every = 8;
  int launched = 0, queued = 0, checked = 0;
  auto gather = [&](CGState *dst) -> hipError_t {
    hipLaunchKernelGGL((kb_gather_states<T>), dim3(unsigned((K + 63) / 64)), dim3(64), 0, st, dj,
                       K, dstates);
    hipError_t e2 = hipGetLastError();
    if (e2 == hipSuccess)
      e2 = hipMemcpyAsync(dst, dstates, size_t(K) * sizeof(CGState), hipMemcpyDeviceToHost, st);
    return e2;
  };
  auto all_done = [&]() {
    bool d = true;
    for (int k = 0; k < K; ++k) d = d && hs[k].done;
    return d;
  };
  // the states before the first chunk
  BTRY(gather(hs.data()));
  BTRY(hipStreamSynchronize(st));
  bool done = all_done();
  while (!done) {
    while (queued - checked < 2 && launched < cg_maxiter) {
      const int batch = cg_maxiter - launched < check_every ? cg_maxiter - launched : check_every;
      for (int q = 0; q < batch; ++q, ++launched) BTRY(iteration(launched & 1));
      const int slot = queued & 1;
      BTRY(gather(hslot + size_t(slot) * K));
      BTRY(hipEventRecord(b->cg_ev[slot], st));
      ++queued;
    }
    if (queued == checked) break;
    const int slot = checked & 1;
    BTRY(hipEventSynchronize(b->cg_ev[slot]));
    std::copy(hslot + size_t(slot) * K, hslot + size_t(slot + 1) * K, hs.begin());
    ++checked;
    done = all_done();
  }
  // chunks still queued return at once (every model's done flag is set, and the states no
  // longer change)
  hipLaunchKernelGGL((kb_update<T, PT>), dim3(unsigned(map_c.size())), dim3(256), 0, st, dj, mc,
                     lr);
  BTRY(hipGetLastError());
  BTRY(hipStreamSynchronize(st));
#undef BTRY
  bool any_nonfinite = false, all_conv = true;
  for (int k = 0; k < K; ++k) {
    nqs_sr_info o;
    fill_info(hs[k], &o);
    any_nonfinite = any_nonfinite || o.status == NQS_ENONFINITE;
    all_conv = all_conv && o.converged;
    if (info) info[k] = o;
  }
  if (any_nonfinite) return NQS_ENONFINITE;
  return all_conv ? NQS_OK : NQS_ENOTCONV;
}

}  // namespace

size_t sr_workspace_bytes(const nqs_model *m, int64_t n) { return sr_layout(m, n).total; }

nqs_status sr_prepare_impl(nqs_model *m, const void *params, const int8_t *sigma, int64_t n,
                           void *ws, size_t ws_bytes, hipStream_t st) {
  if (ws_bytes < sr_layout(m, n).total) return NQS_ENOMEM;
  return m->is_complex ? prepare_impl<true>(m, params, sigma, n, ws, st)
                       : prepare_impl<false>(m, params, sigma, n, ws, st);
}

nqs_status sr_matvec_impl(nqs_model *m, const int8_t *sigma, int64_t n, void *ws,
                          size_t ws_bytes, const void *v, double lambda, void *out,
                          hipStream_t st) {
  if (ws_bytes < sr_layout(m, n).total) return NQS_ENOMEM;
  return m->is_complex ? matvec_impl<true>(m, sigma, n, ws, v, lambda, out, st)
                       : matvec_impl<false>(m, sigma, n, ws, v, lambda, out, st);
}

nqs_status autotune_impl(nqs_model *m, const void *params, const int8_t *sigma, int64_t n,
                         void *ws, size_t ws_bytes, nqs_tune_report *rep, hipStream_t st) {
  SRLayout L = sr_layout(m, n);
  if (ws_bytes < L.total) return NQS_ENOMEM;
  char *b = (char *)ws;
  const int cs = m->is_complex ? 2 : 1;
  const int64_t Pc = (int64_t(m->N) + m->M + int64_t(m->N) * m->M) * cs;
  int cand[NQS_TUNE_MAX];
  int nc = 0;
  const int keep = m->sv_pairs;
  m->sv_pairs = 2;
  const bool pair = grad_plan(m, n).pair;
  cand[nc++] = 2;
  if (pair) cand[nc++] = 4;
  nqs_status s = sr_prepare_impl(m, params, sigma, n, ws, ws_bytes, st);
  if (s != NQS_OK) {
    m->sv_pairs = keep;
    return s;
  }
  hipLaunchKernelGGL(k_fill, dim3(grid_for(Pc)), dim3(256), 0, st, Pc, (double *)(b + L.p), 1.0);
  HIPTRY(hipGetLastError());
  hipEvent_t e0, e1;
  HIPTRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return NQS_EDEVICE;
  }
  double us[NQS_TUNE_MAX] = {0, 0, 0, 0};
  const int reps = 10;
  int best = 0;
  for (int c = 0; c < nc && s == NQS_OK; ++c) {
    m->sv_pairs = cand[c];
    for (int q = 0; q < reps + 2 && s == NQS_OK; ++q) {
      if (q == 2 && hipEventRecord(e0, st) != hipSuccess) s = NQS_EDEVICE;
      if (s == NQS_OK)
        s = sr_matvec_impl(m, sigma, n, ws, ws_bytes, b + L.p, 0.0, b + L.Ap, st);
    }
    float ms = 0.f;
    if (s == NQS_OK && (hipEventRecord(e1, st) != hipSuccess ||
                        hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      s = NQS_EDEVICE;
    us[c] = 1e3 * double(ms) / reps;
    if (us[c] < us[best]) best = c;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  m->sv_pairs = s == NQS_OK ? cand[best] : keep;
  if (rep) {
    rep->n_candidates = nc;
    rep->chosen = best;
    for (int c = 0; c < NQS_TUNE_MAX; ++c) {
      rep->pairs[c] = c < nc ? cand[c] : 0;
      rep->us[c] = c < nc ? us[c] : 0.0;
    }
  }
  return s;
}

nqs_status sr_step_impl(nqs_model *m, void *params, const int8_t *sigma, const void *eloc,
                        int64_t n, int64_t n_chains, double lr, double diag_shift, double cg_tol,
                        int cg_maxiter, void *ws, size_t ws_bytes, nqs_sr_info *info, bool async,
                        hipStream_t st) {
  if (ws_bytes < sr_layout(m, n).total) return NQS_ENOMEM;
  const int64_t nch = n_chains > 0 ? n_chains : n;
#define NQS_SR(T, C)                                                                          \
  (m->ff.L ? sr_ff_impl<T, C>(m, params, sigma, eloc, n, nch, lr, diag_shift, cg_tol,        \
                              cg_maxiter, ws, info, async, st) :                              \
   m->G ? sr_symm_impl<T, C>(m, params, sigma, eloc, n, nch, lr, diag_shift, cg_tol,         \
                             cg_maxiter, ws, info, async, st)                                 \
        : sr_impl<T, C>(m, params, sigma, eloc, n, nch, lr, diag_shift, cg_tol, cg_maxiter,   \
                        ws, info, async, st))
  if (use_double(m)) return m->is_complex ? NQS_SR(double, true) : NQS_SR(double, false);
  return m->is_complex ? NQS_SR(float, true) : NQS_SR(float, false);
#undef NQS_SR
}

size_t batch_sr_workspace_bytes(nqs_batch *b, const int64_t *n_samples) {
  size_t total = 0;
  for (int k = 0; k < b->K; ++k) total += batch_layout(b->models[k], n_samples[k]).total;
  return total;
}

nqs_status batch_sr_step_impl(nqs_batch *b, void *params, const int8_t *samples,
                              const void *eloc, const int64_t *n_samples, const int32_t *n_chains,
                              double lr, double diag_shift, double cg_tol, int cg_maxiter,
                              void *ws, size_t ws_bytes, nqs_sr_info *info, bool async,
                              hipStream_t st) {
  if (ws_bytes < batch_sr_workspace_bytes(b, n_samples)) return NQS_ENOMEM;
  const nqs_model *m = b->models[0];
#define NQS_BSR(T, C)                                                                    \
  batch_sr_impl<T, C>(b, params, samples, eloc, n_samples, n_chains, lr, diag_shift, cg_tol, \
                      cg_maxiter, ws, info, async, st)
  if (use_double(m)) return m->is_complex ? NQS_BSR(double, true) : NQS_BSR(double, false);
  return m->is_complex ? NQS_BSR(float, true) : NQS_BSR(float, false);
#undef NQS_BSR
}
