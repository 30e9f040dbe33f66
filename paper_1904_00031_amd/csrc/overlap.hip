// Supervised learning by the negative log overlap (Sec. 2.2.3, Eq. 1 and Eq. 2).
//
// Direct sampling of the target: cdf_k = sum_{i <= k} |t_i|^2 / max |t|^2 over a training
// set of configurations (one block, fixed summation order), then one thread per draw:
// a Philox uniform u (counter (draw, counter, 0, 3)) picks the first k with
// cdf_k > u cdf_last, and the configuration and log t of row k are gathered.
//
// One SGD step from n target-distributed samples: with d_s = log psi_s - log t_s,
// m = max Re d and R_s = exp(d_s - m) (the common factor exp(m) cancels everywhere),
//   S1 = sum |R_s|^2, S2 = sum conj(R_s),  loss = -log(|S2|^2 / (n S1)),
//   u_s = |R_s|^2 / S1 - conj(R_s) / S2,   g = O^dagger u,   p <- p - lr g.
// The reductions are block partials combined in a fixed order (deterministic); the VJP
// is the Jacobian product of the SR path.
#include "internal.hpp"

namespace {

constexpr int kOvThreads = 256;
constexpr int kOvMaxParts = 1024;

inline unsigned ov_blocks(int64_t n) {
  const int64_t b = (n + kOvThreads - 1) / kOvThreads;
  return unsigned(b < kOvMaxParts ? (b > 0 ? b : 1) : kOvMaxParts);
}

// fixed-order tree sum of one value per thread (blockDim.x = kOvThreads)
__device__ double block_sum(double v, double *sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = kOvThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__device__ double block_max(double v, double *sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = kOvThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// ---- direct sampling of the target --------------------------------------------------

// one block of 1024 threads: thread t owns the contiguous chunk [t c, (t + 1) c)
__global__ __launch_bounds__(1024) void k_target_cdf(int64_t n, int cs, const double *lt,
                                                     double *cdf) {
  __shared__ double sh[1024];
  const int64_t c = (n + 1023) / 1024;
  const int64_t lo = threadIdx.x * c, hi = lo + c < n ? lo + c : n;
  double mx = -INFINITY;
  for (int64_t k = lo; k < hi; ++k) mx = fmax(mx, lt[cs * k]);
  sh[threadIdx.x] = mx;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  const double m = sh[0];
  __syncthreads();
  double acc = 0.0;
  for (int64_t k = lo; k < hi; ++k) acc += exp(2.0 * (lt[cs * k] - m));
  sh[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {  // exclusive prefix of the chunk sums, in order
    double run = 0.0;
    for (int t = 0; t < 1024; ++t) {
      const double v = sh[t];
      sh[t] = run;
      run += v;
    }
  }
  __syncthreads();
  double run = sh[threadIdx.x];
  for (int64_t k = lo; k < hi; ++k) {
    run += exp(2.0 * (lt[cs * k] - m));
    cdf[k] = run;
  }
}

__global__ void k_target_draw(int64_t n_states, const double *__restrict__ cdf, int N,
                              const int8_t *__restrict__ states, int cs,
                              const double *__restrict__ lt, int64_t n, uint32_t k0,
                              uint32_t k1, uint32_t counter, int8_t *__restrict__ sigma,
                              double *__restrict__ lt_out, int64_t *__restrict__ index) {
  for (int64_t s = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; s < n;
       s += int64_t(gridDim.x) * blockDim.x) {
    const Philox4 w = philox4x32_10(uint32_t(s), counter, 0u, TAG_TARGET, k0, k1);
    const double x = rng_uniform(w.w[1], w.w[2]) * cdf[n_states - 1];
    int64_t lo = 0, hi = n_states - 1;   // first k with cdf[k] > x (x < cdf_last)
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo) / 2;
      if (cdf[mid] > x)
        hi = mid;
      else
        lo = mid + 1;
    }
    if (index) index[s] = lo;
    for (int c = 0; c < cs; ++c) lt_out[cs * s + c] = lt[cs * lo + c];
    for (int i = 0; i < N; ++i) sigma[s * N + i] = states[lo * N + i];
  }
}

// ---- the overlap step ---------------------------------------------------------------

struct OvState {
  double m, S1, S2r, S2i, loss;
  int finite;
};

__global__ __launch_bounds__(kOvThreads) void k_ov_max(int64_t n, int cs, const double *lp,
                                                       const double *lt, double *part) {
  __shared__ double sh[kOvThreads];
  double mx = -INFINITY;
  for (int64_t s = blockIdx.x * int64_t(kOvThreads) + threadIdx.x; s < n;
       s += int64_t(gridDim.x) * kOvThreads)
    mx = fmax(mx, lp[cs * s] - lt[cs * s]);
  mx = block_max(mx, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = mx;
}

// every block reduces the max partials itself (same order, same result), then its sums
__global__ __launch_bounds__(kOvThreads) void k_ov_sums(int64_t n, int cs, const double *lp,
                                                        const double *lt, const double *pmax,
                                                        int nparts, double *part) {
  __shared__ double sh[kOvThreads];
  double mx = -INFINITY;
  for (int k = threadIdx.x; k < nparts; k += kOvThreads) mx = fmax(mx, pmax[k]);
  const double m = block_max(mx, sh);
  double s1 = 0.0, s2r = 0.0, s2i = 0.0;
  for (int64_t s = blockIdx.x * int64_t(kOvThreads) + threadIdx.x; s < n;
       s += int64_t(gridDim.x) * kOvThreads) {
    const double dr = lp[cs * s] - lt[cs * s] - m;
    const double di = cs == 2 ? lp[2 * s + 1] - lt[2 * s + 1] : 0.0;
    const double e = exp(dr);
    s1 += e * e;
    s2r += e * cos(di);
    s2i -= e * sin(di);
  }
  s1 = block_sum(s1, sh);
  s2r = block_sum(s2r, sh);
  s2i = block_sum(s2i, sh);
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x] = s1;
    part[3 * blockIdx.x + 1] = s2r;
    part[3 * blockIdx.x + 2] = s2i;
    if (blockIdx.x == 0) part[3 * kOvMaxParts] = m;
  }
}

__global__ __launch_bounds__(kOvThreads) void k_ov_finish(int64_t n, int nparts,
                                                          const double *part, OvState *st) {
  __shared__ double sh[kOvThreads];
  double s1 = 0.0, s2r = 0.0, s2i = 0.0;
  for (int k = threadIdx.x; k < nparts; k += kOvThreads) {
    s1 += part[3 * k];
    s2r += part[3 * k + 1];
    s2i += part[3 * k + 2];
  }
  s1 = block_sum(s1, sh);
  s2r = block_sum(s2r, sh);
  s2i = block_sum(s2i, sh);
  if (threadIdx.x == 0) {
    OvState o;
    o.m = part[3 * kOvMaxParts];
    o.S1 = s1;
    o.S2r = s2r;
    o.S2i = s2i;
    o.loss = -log((s2r * s2r + s2i * s2i) / (double(n) * s1));
    o.finite = isfinite(o.m) && isfinite(s1) && s1 > 0.0 && isfinite(s2r) && isfinite(s2i) &&
               isfinite(o.loss);
    *st = o;
  }
}

__global__ void k_ov_u(int64_t n, int cs, const double *lp, const double *lt,
                       const OvState *st, double *u) {
  const OvState o = *st;
  const double den = o.S2r * o.S2r + o.S2i * o.S2i;
  for (int64_t s = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; s < n;
       s += int64_t(gridDim.x) * blockDim.x) {
    const double dr = lp[cs * s] - lt[cs * s] - o.m;
    const double e = exp(dr);
    if (cs == 2) {
      const double di = lp[2 * s + 1] - lt[2 * s + 1];
      const double cr = e * cos(di), ci = -e * sin(di);   // conj(R)
      // conj(R) / S2
      const double qr = (cr * o.S2r + ci * o.S2i) / den, qi = (ci * o.S2r - cr * o.S2i) / den;
      u[2 * s] = e * e / o.S1 - qr;
      u[2 * s + 1] = -qi;
    } else {
      u[s] = e * e / o.S1 - e / o.S2r;
    }
  }
}

// p <- p - lr g when the loss and the gradient are finite
template <typename PT>
__global__ void k_ov_update(int64_t Pc, PT *params, const double *g, double lr,
                            const OvState *st, const double *gn) {
  if (!st->finite || !isfinite(*gn)) return;
  for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < Pc;
       k += int64_t(gridDim.x) * blockDim.x)
    params[k] = PT(double(params[k]) - lr * g[k]);
}

// ||g||_2 in a fixed order (one block)
__global__ __launch_bounds__(kOvThreads) void k_ov_gnorm(int64_t Pc, const double *g,
                                                         double *out) {
  __shared__ double sh[kOvThreads];
  double a = 0.0;
  for (int64_t k = threadIdx.x; k < Pc; k += kOvThreads) a += g[k] * g[k];
  a = block_sum(a, sh);
  if (threadIdx.x == 0) *out = sqrt(a);
}

}  // namespace

hipError_t launch_target_cdf(const nqs_model *m, const void *log_t, int64_t n_states,
                             double *cdf, hipStream_t st) {
  hipLaunchKernelGGL(k_target_cdf, dim3(1), dim3(1024), 0, st, n_states,
                     m->is_complex ? 2 : 1, (const double *)log_t, cdf);
  return hipGetLastError();
}

hipError_t launch_target_draw(const nqs_model *m, const double *cdf, int64_t n_states,
                              const int8_t *states, const void *log_t, int64_t n,
                              uint64_t seed, uint64_t counter, int8_t *sigma, void *log_t_out,
                              int64_t *index, hipStream_t st) {
  const int64_t b = (n + 255) / 256;
  hipLaunchKernelGGL(k_target_draw, dim3(unsigned(b < 65536 ? b : 65536)), dim3(256), 0, st,
                     n_states, cdf, m->N, states, m->is_complex ? 2 : 1, (const double *)log_t,
                     n, uint32_t(seed & 0xffffffffu), uint32_t(seed >> 32), uint32_t(counter),
                     sigma, (double *)log_t_out, index);
  return hipGetLastError();
}

// the Jacobian scratch of the model's ansatz (RBM or FFNN) at the start of the scratch
size_t jac_bytes(const nqs_model *m, int64_t n) {
  return m->ff.L ? ff_grad_scratch_bytes(m, n) : grad_scratch_bytes(m, n);
}

size_t overlap_scratch_bytes(const nqs_model *m, int64_t n) {
  const size_t cs = m->is_complex ? 2 : 1;
  auto r = [](size_t b) { return (b + 255) / 256 * 256; };
  return r(jac_bytes(m, n)) + r(cs * 8 * size_t(n)) * 2 +
         r(cs * 8 * size_t(n_params_model(m))) + r(8 * (4 * kOvMaxParts + 1)) +
         r(sizeof(OvState)) + 256;
}

nqs_status overlap_step_impl(nqs_model *m, void *params, const int8_t *sigma,
                             const void *log_t, int64_t n, double lr, void *scratch,
                             nqs_overlap_info *info, hipStream_t st) {
  const int cs = m->is_complex ? 2 : 1;
  auto r = [](size_t b) { return (b + 255) / 256 * 256; };
  char *base = (char *)scratch;
  size_t off = r(jac_bytes(m, n));
  double *lp = (double *)(base + off);
  off += r(cs * 8 * size_t(n));
  double *u = (double *)(base + off);
  off += r(cs * 8 * size_t(n));
  double *g = (double *)(base + off);
  off += r(cs * 8 * size_t(n_params_model(m)));
  double *part = (double *)(base + off);          // [2 kOvMaxParts] max, [3 kOvMaxParts + 1]
  off += r(8 * (4 * kOvMaxParts + 1));
  OvState *state = (OvState *)(base + off);
  off += r(sizeof(OvState));
  double *gn = (double *)(base + off);
  const int64_t Pc = cs * n_params_model(m);

  hipError_t e = hipSuccess;
  const bool ff = m->ff.L > 0;
  const void *pe = ff ? params : model_params(m, params, st, &e);
  if (e == hipSuccess) e = ff ? launch_ff_tables(m, pe, st) : launch_tables(m, pe, st);
  if (e == hipSuccess)
    e = ff ? launch_ff_log_psi(m, pe, sigma, n, lp, st) : launch_log_psi(m, sigma, n, lp, st);
  const unsigned nb = ov_blocks(n);
  double *pmax = part + 3 * kOvMaxParts + 1;
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_ov_max, dim3(nb), dim3(kOvThreads), 0, st, n, cs, lp,
                       (const double *)log_t, pmax);
    hipLaunchKernelGGL(k_ov_sums, dim3(nb), dim3(kOvThreads), 0, st, n, cs, lp,
                       (const double *)log_t, pmax, int(nb), part);
    hipLaunchKernelGGL(k_ov_finish, dim3(1), dim3(kOvThreads), 0, st, n, int(nb), part, state);
    hipLaunchKernelGGL(k_ov_u, dim3(nb), dim3(kOvThreads), 0, st, n, cs, lp,
                       (const double *)log_t, state, u);
    e = hipGetLastError();
  }
  if (ff) {
    if (e == hipSuccess) e = launch_ff_fb(m, pe, sigma, n, scratch, st);
    if (e == hipSuccess) e = launch_ff_vjp(m, sigma, n, u, scratch, g, nullptr, st);
  } else {
    if (e == hipSuccess) e = launch_theta_tanh(m, sigma, n, scratch, true, st);
    if (e == hipSuccess) e = launch_vjp_partials(m, sigma, n, u, scratch, nullptr, st);
    if (e == hipSuccess) e = launch_vjp_reduce(m, n, scratch, m->G ? m->d_gexp : g, nullptr, st);
    if (e == hipSuccess && m->G) e = launch_symm_reduce(m, m->d_gexp, g, st);
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_ov_gnorm, dim3(1), dim3(kOvThreads), 0, st, Pc, g, gn);
    if (use_double(m))
      hipLaunchKernelGGL(k_ov_update<double>, dim3(ov_blocks(Pc)), dim3(kOvThreads), 0, st, Pc,
                         (double *)params, g, lr, state, gn);
    else
      hipLaunchKernelGGL(k_ov_update<float>, dim3(ov_blocks(Pc)), dim3(kOvThreads), 0, st, Pc,
                         (float *)params, g, lr, state, gn);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return NQS_EDEVICE;
  OvState h;
  double hg = 0.0;
  e = hipMemcpyAsync(&h, state, sizeof h, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(&hg, gn, sizeof hg, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return NQS_EDEVICE;
  const bool ok = h.finite && std::isfinite(hg);
  if (info) {
    info->loss = h.loss;
    info->overlap = exp(-h.loss);
    info->grad_norm = hg;
    info->status = ok ? NQS_OK : NQS_ENONFINITE;
    info->reserved = 0;
  }
  return ok ? NQS_OK : NQS_ENONFINITE;
}
