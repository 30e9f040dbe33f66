// The symmetric RBM (RbmSpinSymm, Sec. 2.2.2): alpha filters shared over a group of G
// site permutations. Its amplitude is that of a plain RBM with M = alpha G hidden units
// whose parameters are the expansion E p of the symmetric ones,
//   a_i = a,  b_(fG+g) = b_f,  W_(fG+g), perm[g][i] = W_f,i,
// so every kernel of the plain RBM runs unchanged on E p. The Jacobian follows from the
// chain rule: O_sym = O_exp E, hence O_sym v = O_exp (E v) and O_sym^dagger u =
// E^T (O_exp^dagger u), where E^T sums the copies of each symmetric parameter.
#include "internal.hpp"

namespace {

inline unsigned blocks_for(int64_t count) {
  const int64_t b = (count + 255) / 256;
  return unsigned(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

// one thread per element of the expanded parameters; W elements are enumerated as
// (unit j, symmetric column i) and scattered to column perm[g][i] (a permutation: every
// expanded element is written once)
template <typename PT, bool C>
__global__ void k_symm_expand(int N, int G, int alpha, const int *__restrict__ perm,
                              const PT *__restrict__ ps, PT *__restrict__ pe,
                              const int *skip) {
  if (skip && *skip) return;
  constexpr int cs = C ? 2 : 1;
  const int M = alpha * G;
  const int64_t total = int64_t(N) + M + int64_t(M) * N;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    int64_t src, dst;
    if (e < N) {
      src = 0;
      dst = e;
    } else if (e < N + M) {
      const int j = int(e - N);
      src = 1 + j / G;
      dst = e;
    } else {
      const int64_t q = e - N - M;
      const int j = int(q / N), i = int(q % N);
      const int f = j / G, g = j % G;
      src = 1 + alpha + int64_t(f) * N + i;
      dst = int64_t(N) + M + int64_t(j) * N + perm[int64_t(g) * N + i];
    }
#pragma unroll
    for (int c = 0; c < cs; ++c) pe[cs * dst + c] = ps[cs * src + c];
  }
}

// one thread per symmetric parameter: the sum of its copies in a fixed order
template <bool C>
__global__ void k_symm_reduce(int N, int G, int alpha, const int *__restrict__ perm,
                              const double *__restrict__ ge, double *__restrict__ gs) {
  constexpr int cs = C ? 2 : 1;
  const int M = alpha * G;
  const int64_t P = 1 + alpha + int64_t(alpha) * N;
  for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < P;
       k += int64_t(gridDim.x) * blockDim.x) {
    double acc[cs];
#pragma unroll
    for (int c = 0; c < cs; ++c) acc[c] = 0.0;
    if (k == 0) {
      for (int i = 0; i < N; ++i)
#pragma unroll
        for (int c = 0; c < cs; ++c) acc[c] += ge[cs * int64_t(i) + c];
    } else if (k <= alpha) {
      const int f = int(k - 1);
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int c = 0; c < cs; ++c) acc[c] += ge[cs * (int64_t(N) + f * G + g) + c];
    } else {
      const int64_t q = k - 1 - alpha;
      const int f = int(q / N), i = int(q % N);
      for (int g = 0; g < G; ++g) {
        const int64_t e = int64_t(N) + M + int64_t(f * G + g) * N + perm[int64_t(g) * N + i];
#pragma unroll
        for (int c = 0; c < cs; ++c) acc[c] += ge[cs * e + c];
      }
    }
#pragma unroll
    for (int c = 0; c < cs; ++c) gs[cs * k + c] = acc[c];
  }
}

}  // namespace

hipError_t launch_symm_expand(const nqs_model *m, const void *p_sym, void *p_exp,
                              hipStream_t st) {
  const unsigned g = blocks_for(n_params_exp(m));
  if (use_double(m)) {
    if (m->is_complex)
      hipLaunchKernelGGL((k_symm_expand<double, true>), dim3(g), dim3(256), 0, st, m->N, m->G,
                         m->alpha, m->d_perm, (const double *)p_sym, (double *)p_exp, nullptr);
    else
      hipLaunchKernelGGL((k_symm_expand<double, false>), dim3(g), dim3(256), 0, st, m->N, m->G,
                         m->alpha, m->d_perm, (const double *)p_sym, (double *)p_exp, nullptr);
  } else {
    if (m->is_complex)
      hipLaunchKernelGGL((k_symm_expand<float, true>), dim3(g), dim3(256), 0, st, m->N, m->G,
                         m->alpha, m->d_perm, (const float *)p_sym, (float *)p_exp, nullptr);
    else
      hipLaunchKernelGGL((k_symm_expand<float, false>), dim3(g), dim3(256), 0, st, m->N, m->G,
                         m->alpha, m->d_perm, (const float *)p_sym, (float *)p_exp, nullptr);
  }
  return hipGetLastError();
}

hipError_t launch_symm_expand_dir(const nqs_model *m, const double *v_sym, double *v_exp,
                                  const int *skip, hipStream_t st) {
  const unsigned g = blocks_for(n_params_exp(m));
  if (m->is_complex)
    hipLaunchKernelGGL((k_symm_expand<double, true>), dim3(g), dim3(256), 0, st, m->N, m->G,
                       m->alpha, m->d_perm, v_sym, v_exp, skip);
  else
    hipLaunchKernelGGL((k_symm_expand<double, false>), dim3(g), dim3(256), 0, st, m->N, m->G,
                       m->alpha, m->d_perm, v_sym, v_exp, skip);
  return hipGetLastError();
}

hipError_t launch_symm_reduce(const nqs_model *m, const double *g_exp, double *g_sym,
                              hipStream_t st) {
  const unsigned g = blocks_for(n_params_model(m));
  if (m->is_complex)
    hipLaunchKernelGGL((k_symm_reduce<true>), dim3(g), dim3(256), 0, st, m->N, m->G, m->alpha,
                       m->d_perm, g_exp, g_sym);
  else
    hipLaunchKernelGGL((k_symm_reduce<false>), dim3(g), dim3(256), 0, st, m->N, m->G, m->alpha,
                       m->d_perm, g_exp, g_sym);
  return hipGetLastError();
}

const void *model_params(nqs_model *m, const void *p, hipStream_t st, hipError_t *err) {
  *err = hipSuccess;
  if (!m->G) return p;
  *err = launch_symm_expand(m, p, m->d_pexp, st);
  return m->d_pexp;
}
