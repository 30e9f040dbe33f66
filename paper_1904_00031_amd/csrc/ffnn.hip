// The feed-forward network (FFNN, Sec. 2.2.2): L dense layers, each followed by ln cosh
// or tanh, log psi = sum of the last layer's outputs.
//
//   z_0 = sigma,  y_l = W_l z_l + b_l (layer l maps w[l] -> w[l+1]),  z_(l+1) = f_l(y_l)
//
// One wavefront per configuration: lane t owns the outputs j = t + 64 r of a layer
// (r < 8, widths <= 512), the layer's input row sits in LDS and is read as a broadcast,
// and W_l is read transposed ([w[l]][w[l+1]], a table refreshed per call) so that the
// lanes of a wavefront read consecutive elements. Sampling and local energies keep the
// first layer's angles theta = W_0 sigma + b_0 in double in registers and update them
// by the columns of W_0 a move changes, as for the RBM; the later layers are evaluated
// in full for every proposal and connected configuration.
//
// Log-derivatives (backpropagation): with g_l = d log psi / d y_l, g_(L-1) = f'(y_(L-1))
// and g_l = f'(y_l) * (W_(l+1)^T g_(l+1)); O_(b_l) = g_l and O_(W_l),jk = g_l,j z_l,k.
// A forward and backward pass stores the rows Z (the inputs z_1 .. z_(L-1)) and G (every
// g_l) of each sample; then
//   (O v)_s          = sum_l sum_j g_l,j (vb_l,j + sum_k vW_l,jk z_l,k)      (per sample)
//   (O^dagger u)_jk  = sum_s conj(g_l,sj z_l,sk) u_s                         (over samples)
// the second as 64 x 64 output tiles over sample splits (partials in the compute
// precision, summed over the splits in a fixed order in double).
#include "internal.hpp"

namespace {

constexpr int kFfR = kFfMaxWidth / 64;   // output chunks of 64 per lane

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

template <typename T, bool C>
__device__ __forceinline__ V<T, C> ff_act(int a, V<T, C> y) {
  return a == NQS_ACT_LNCOSH ? vlncosh<T, C>(y) : vtanh<T, C>(y);
}

// f'(y): tanh y for ln cosh, 1 - tanh^2 y for tanh
template <typename T, bool C>
__device__ __forceinline__ V<T, C> ff_dact(int a, V<T, C> y) {
  const V<T, C> t = vtanh<T, C>(y);
  return a == NQS_ACT_LNCOSH ? t : vsub(vmake<T, C>(T(1), T(0)), vmul(t, t));
}

// b + sum_(k < wi) W[k stride + j] z_k: the weights loaded eight at a time, four partial
// sums (k mod 4) added in a fixed order at the end (short dependency chains for the one
// wavefront that evaluates a configuration)
template <typename T, bool C>
__device__ __forceinline__ V<T, C> ff_dot(V<T, C> b, const T *__restrict__ W, int64_t stride,
                                          int j, const T *z, int wi) {
  V<T, C> a[4] = {b, vmake<T, C>(T(0), T(0)), vmake<T, C>(T(0), T(0)),
                  vmake<T, C>(T(0), T(0))};
  int k = 0;
  for (; k + 8 <= wi; k += 8) {
    V<T, C> wv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) wv[q] = vload<T, C>(W, int64_t(k + q) * stride + j);
#pragma unroll
    for (int q = 0; q < 8; ++q) a[q & 3] = vadd(a[q & 3], vmul(wv[q], vload<T, C>(z, k + q)));
  }
  for (; k < wi; ++k) a[0] = vadd(a[0], vmul(vload<T, C>(W, int64_t(k) * stride + j), vload<T, C>(z, k)));
  return vadd(vadd(a[0], a[1]), vadd(a[2], a[3]));
}

// Layers l0 .. L-1 of one configuration whose layer-l0 input is in zi (LDS); zo is the
// other LDS buffer. zrow / grow (may be NULL): global Z and G rows that receive the layer
// inputs and f'(y_l). Wt holds the transposed weights from table offset tbase on (the
// whole table in global memory, or layers 1.. staged in LDS). Returns the wave-uniform sum
// of the last layer's outputs.
template <typename T, bool C>
__device__ V<double, C> ff_layers(const FfDev &f, const T *__restrict__ P,
                                  const T *__restrict__ Wt, int64_t tbase, int l0, T *zi, T *zo,
                                  int lane, T *zrow, T *grow) {
  constexpr int cs = C ? 2 : 1;
  double tr = 0.0, ti = 0.0;
  for (int l = l0; l < f.L; ++l) {
    const int wi = f.w[l], wo = f.w[l + 1];
    const int nr = (wo + 63) >> 6;
    const T *W = Wt + cs * (f.toff[l] - tbase);
    for (int r = 0; r < nr; ++r) {
      const int j = lane + 64 * r;
      const int jc = j < wo ? j : wo - 1;
      const V<T, C> acc = ff_dot<T, C>(vload<T, C>(P, f.poff[l] + jc), W, wo, jc, zi, wi);
      if (j < wo) {
        if (grow) vstore(grow, f.goff[l] + j, ff_dact<T, C>(f.act[l], acc));
        const V<T, C> z = ff_act<T, C>(f.act[l], acc);
        if (l + 1 < f.L) {
          vstore(zo, j, z);
          if (zrow) vstore(zrow, f.zoff[l + 1] + j, z);
        } else {
          tr += double(z.re);
          ti += double(z.im);
        }
      }
    }
    wave_sync();
    T *tmp = zi;
    zi = zo;
    zo = tmp;
  }
  return vmake<double, C>(wave_sum(tr), C ? wave_sum(ti) : 0.0);
}

// log psi from first-layer angles th (lane units j = lane + 64 r of layer 0); Wl: the
// weights of layers 1.. (table offset toff[1] on)
template <typename T, bool C>
__device__ V<double, C> ff_from_theta(const FfDev &f, const T *__restrict__ P,
                                      const T *__restrict__ Wl, const V<double, C> *th, T *zi,
                                      T *zo, int lane) {
  const int w1 = f.w[1];
  double tr = 0.0, ti = 0.0;
#pragma unroll
  for (int r = 0; r < kFfR; ++r) {
    const int j = lane + 64 * r;
    if (j < w1) {
      const V<T, C> z = ff_act<T, C>(f.act[0], vmake<T, C>(T(th[r].re), T(th[r].im)));
      if (f.L > 1) {
        vstore(zi, j, z);
      } else {
        tr += double(z.re);
        ti += double(z.im);
      }
    }
  }
  if (f.L == 1) return vmake<double, C>(wave_sum(tr), C ? wave_sum(ti) : 0.0);
  wave_sync();
  return ff_layers<T, C>(f, P, Wl, f.toff[1], 1, zi, zo, lane, nullptr, nullptr);
}

// theta = W_0 sigma + b_0 in double from the spins in LDS
template <typename T, bool C>
__device__ void ff_theta(const FfDev &f, const T *__restrict__ P, const T *__restrict__ Wt,
                         const int8_t *sig, int lane, V<double, C> *th) {
  constexpr int cs = C ? 2 : 1;
  const int w1 = f.w[1];
#pragma unroll
  for (int r = 0; r < kFfR; ++r) {
    const int j = lane + 64 * r;
    th[r] = vmake<double, C>(0.0, 0.0);
    if (j < w1) {
      V<double, C> acc = vload<double, C>(P, f.poff[0] + j);
      for (int i = 0; i < f.N; ++i) {
        const double s = double(sig[i]);
        const V<double, C> w = vload<double, C>(Wt, int64_t(i) * w1 + j);
        acc.re += s * w.re;
        if (C) acc.im += s * w.im;
      }
      th[r] = acc;
    }
  }
  (void)cs;
}

// th2 = th - 2 s_i W_0[:, i] (- 2 s_k W_0[:, k] when k >= 0)
template <typename T, bool C>
__device__ __forceinline__ void ff_move(const FfDev &f, const T *__restrict__ Wt,
                                        const V<double, C> *th, int i, double si, int k,
                                        double sk, int lane, V<double, C> *th2) {
  const int w1 = f.w[1];
#pragma unroll
  for (int r = 0; r < kFfR; ++r) {
    const int j = lane + 64 * r;
    th2[r] = th[r];
    if (j < w1) {
      const V<double, C> a = vload<double, C>(Wt, int64_t(i) * w1 + j);
      th2[r].re -= 2.0 * si * a.re;
      if (C) th2[r].im -= 2.0 * si * a.im;
      if (k >= 0) {
        const V<double, C> b = vload<double, C>(Wt, int64_t(k) * w1 + j);
        th2[r].re -= 2.0 * sk * b.re;
        if (C) th2[r].im -= 2.0 * sk * b.im;
      }
    }
  }
}

struct FfWave {
  int Npad, zbytes;   // spins (padded) and one z buffer, bytes
  __host__ __device__ int bytes() const { return Npad + 2 * zbytes; }
};

// The weights of layers 1.. (table elements toff[1] .. tab) copied into LDS after the
// wavefronts' buffers (wpb of them) by the whole block; returns that copy
template <typename T, bool C>
__device__ __forceinline__ const T *ff_stage_layers(const FfDev &f, FfWave fw, int wpb,
                                                    const T *__restrict__ Wt) {
  extern __shared__ __align__(16) unsigned char ff_lds[];
  constexpr int cs = C ? 2 : 1;
  T *dst = reinterpret_cast<T *>(ff_lds + int64_t(wpb) * fw.bytes());
  const int64_t n = int64_t(cs) * (f.tab - f.toff[1]);
  const T *src = Wt + int64_t(cs) * f.toff[1];
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) dst[e] = src[e];
  __syncthreads();
  return dst;
}

template <typename T, bool C>
__device__ __forceinline__ void ff_wave_ptrs(FfWave fw, int wid, int8_t **sig, T **za, T **zb) {
  extern __shared__ __align__(16) unsigned char ff_lds[];
  unsigned char *base = ff_lds + int64_t(wid) * fw.bytes();
  *sig = reinterpret_cast<int8_t *>(base);
  *za = reinterpret_cast<T *>(base + fw.Npad);
  *zb = reinterpret_cast<T *>(base + fw.Npad + fw.zbytes);
}

// W_l transposed into the table (compute precision)
template <typename T, bool C>
__global__ void k_ff_tables(FfDev f, const T *__restrict__ P, T *__restrict__ Wt) {
  for (int l = 0; l < f.L; ++l) {
    const int wi = f.w[l], wo = f.w[l + 1];
    const int64_t tot = int64_t(wi) * wo;
    for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < tot;
         e += int64_t(gridDim.x) * blockDim.x) {
      const int64_t k = e / wo, j = e % wo;   // Wt[k][j] = W[j][k]
      vstore(Wt, f.toff[l] + e, vload<T, C>(P, f.poff[l] + wo + j * wi + k));
    }
  }
}

// log psi of every configuration (one wavefront each)
template <typename T, bool C>
__global__ __launch_bounds__(256) void k_ff_log_psi(FfDev f, FfWave fw, const T *P,
                                                    const T *Wt, const int8_t *sigma,
                                                    int64_t n, double *out) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int8_t *sig;
  T *za, *zb;
  ff_wave_ptrs<T, C>(fw, wid, &sig, &za, &zb);
  const int64_t waves = int64_t(gridDim.x) * (blockDim.x >> 6);
  for (int64_t s = int64_t(blockIdx.x) * (blockDim.x >> 6) + wid; s < n; s += waves) {
    for (int i = lane; i < f.N; i += 64) vstore(za, i, vmake<T, C>(T(sigma[s * f.N + i]), T(0)));
    wave_sync();
    const V<double, C> lp = ff_layers<T, C>(f, P, Wt, 0, 0, za, zb, lane, nullptr, nullptr);
    if (lane == 0) vstore(out, s, lp);
    wave_sync();
  }
}

// E_loc (Eq. 5) of every configuration from the ratios psi(sigma') / psi(sigma)
template <typename T, bool C, bool WL>
__global__ __launch_bounds__(256) void k_ff_eloc(FfDev f, FfWave fw, DevModel dm, const T *P,
                                                 const T *Wt, const int8_t *sigma, int64_t n,
                                                 double *eloc) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int8_t *sig;
  T *za, *zb;
  ff_wave_ptrs<T, C>(fw, wid, &sig, &za, &zb);
  constexpr int cs = C ? 2 : 1;
  const T *Wl = WL ? ff_stage_layers<T, C>(f, fw, int(blockDim.x >> 6), Wt)
                   : Wt + int64_t(cs) * f.toff[1];
  const bool tfim = dm.ham == NQS_TFIM;
  const int64_t waves = int64_t(gridDim.x) * (blockDim.x >> 6);
  V<double, C> th[kFfR], th2[kFfR];
  for (int64_t s = int64_t(blockIdx.x) * (blockDim.x >> 6) + wid; s < n; s += waves) {
    for (int i = lane; i < f.N; i += 64) sig[i] = sigma[s * f.N + i];
    wave_sync();
    ff_theta<T, C>(f, P, Wt, sig, lane, th);
    const V<double, C> lp = ff_from_theta<T, C>(f, P, Wl, th, za, zb, lane);
    double diag = 0.0;
    for (int b = lane; b < dm.Btot; b += 64)
      diag += dm.bond_diag[b] * double(sig[dm.bonds[2 * b]]) * double(sig[dm.bonds[2 * b + 1]]);
    diag = wave_sum(diag);
    double er = diag, ei = 0.0;
    const int ncand = tfim ? (dm.h != 0.0 ? f.N : 0) : dm.Btot;
    for (int c = 0; c < ncand; ++c) {
      int i, k;
      double el;
      if (tfim) {
        i = c;
        k = -1;
        el = -dm.h;
      } else {
        i = dm.bonds[2 * c];
        k = dm.bonds[2 * c + 1];
        el = dm.bond_off[c];
        if (sig[i] == sig[k] || el == 0.0) continue;
      }
      ff_move<T, C>(f, Wt, th, i, double(sig[i]), k, k >= 0 ? double(sig[k]) : 0.0, lane, th2);
      const V<double, C> lq = ff_from_theta<T, C>(f, P, Wl, th2, za, zb, lane);
      const double e = exp(lq.re - lp.re);
      if (C) {
        double sn, cn;
        sincos(lq.im - lp.im, &sn, &cn);
        er += el * e * cn;
        ei += el * e * sn;
      } else {
        er += el * e;
      }
    }
    if (lane == 0) {
      if (C) {
        eloc[2 * s] = er;
        eloc[2 * s + 1] = ei;
      } else {
        eloc[s] = er;
      }
    }
    wave_sync();
  }
}

struct FfSweepArgs {
  int8_t *chain_sigma;
  int n_chains, n_sweeps, n_discard;
  uint32_t k0, k1, counter, chain_offset;
  int8_t *samples;
  int64_t *n_acc;
};

// Metropolis sweeps (Sec. 2.2.5) of one chain per wavefront: the proposal stream, the
// identity exchange and the accept rule of the RBM sweep; the ratio from log psi of the
// proposed configuration, evaluated from the updated first-layer angles, in double for
// FP64 models and through the FP32 layers otherwise
template <typename T, bool C, bool WL>
__global__ __launch_bounds__(256) void k_ff_sweep(FfDev f, FfWave fw, DevModel dm, const T *P,
                                                  const T *Wt, FfSweepArgs a) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int chain = blockIdx.x * (blockDim.x >> 6) + wid;
  constexpr int cs = C ? 2 : 1;
  // (the staging barrier comes before any wavefront leaves)
  const T *Wl = WL ? ff_stage_layers<T, C>(f, fw, int(blockDim.x >> 6), Wt)
                   : Wt + int64_t(cs) * f.toff[1];
  if (chain >= a.n_chains) return;
  int8_t *sig;
  T *za, *zb;
  ff_wave_ptrs<T, C>(fw, wid, &sig, &za, &zb);
  const int N = f.N;
  const bool flip = dm.move == NQS_MOVE_FLIP;
  for (int i = lane; i < N; i += 64) sig[i] = a.chain_sigma[int64_t(chain) * N + i];
  wave_sync();
  V<double, C> th[kFfR], th2[kFfR];
  ff_theta<T, C>(f, P, Wt, sig, lane, th);
  V<double, C> lp = ff_from_theta<T, C>(f, P, Wl, th, za, zb, lane);
  const uint32_t cid = a.chain_offset + uint32_t(chain);
  int64_t acc_count = 0;
  const int total = a.n_discard + a.n_sweeps;
  for (int sw = 0; sw < total; ++sw) {
    for (int st = 0; st < N; ++st) {
      const Philox4 w = philox4x32_10(cid, a.counter + uint32_t(sw), uint32_t(st), TAG_PROPOSAL,
                                      a.k0, a.k1);
      int i, k;
      if (flip) {
        i = rng_index(w.w[0], uint32_t(N));
        k = -1;
      } else {
        const int row = rng_index(w.w[0], uint32_t(dm.B0));
        i = dm.bonds[2 * row];
        k = dm.bonds[2 * row + 1];
      }
      const double u = rng_uniform(w.w[1], w.w[2]);
      const int si = sig[i];
      const int sk = k >= 0 ? sig[k] : 0;
      if (!flip && si == sk) continue;   // an exchange of equal spins is the identity move
      ff_move<T, C>(f, Wt, th, i, double(si), k, double(sk), lane, th2);
      const V<double, C> lq = ff_from_theta<T, C>(f, P, Wl, th2, za, zb, lane);
      const double ex = 2.0 * (lq.re - lp.re);
      const int accept = __builtin_amdgcn_readfirstlane(int(ex >= 0.0 || u < exp(ex)));
      if (accept) {
#pragma unroll
        for (int r = 0; r < kFfR; ++r) th[r] = th2[r];
        lp = lq;
        wave_sync();
        if (lane == 0) {
          sig[i] = int8_t(-si);
          if (k >= 0) sig[k] = int8_t(-sk);
        }
        wave_sync();
        ++acc_count;
      }
    }
    if (sw >= a.n_discard) {
      int8_t *dst = a.samples + (int64_t(sw - a.n_discard) * a.n_chains + chain) * N;
      for (int i = lane; i < N; i += 64) dst[i] = sig[i];
    }
  }
  for (int i = lane; i < N; i += 64) a.chain_sigma[int64_t(chain) * N + i] = sig[i];
  if (lane == 0 && a.n_acc) a.n_acc[chain] = acc_count;
}

// forward and backward pass: Z rows (z_1 .. z_(L-1)) and G rows (g_0 .. g_(L-1))
template <typename T, bool C>
__global__ __launch_bounds__(256) void k_ff_fb(FfDev f, FfWave fw, const T *P, const T *Wt,
                                               const int8_t *sigma, int64_t n, T *Z, T *G) {
  constexpr int cs = C ? 2 : 1;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int8_t *sig;
  T *za, *zb;
  ff_wave_ptrs<T, C>(fw, wid, &sig, &za, &zb);
  const int64_t waves = int64_t(gridDim.x) * (blockDim.x >> 6);
  for (int64_t s = int64_t(blockIdx.x) * (blockDim.x >> 6) + wid; s < n; s += waves) {
    T *zrow = Z + int64_t(cs) * s * f.zcols;
    T *grow = G + int64_t(cs) * s * f.gcols;
    for (int i = lane; i < f.N; i += 64) vstore(za, i, vmake<T, C>(T(sigma[s * f.N + i]), T(0)));
    wave_sync();
    ff_layers<T, C>(f, P, Wt, 0, 0, za, zb, lane, zrow, grow);
    // backward: g_l = f'(y_l) * (W_(l+1)^T g_(l+1)); every lane reads back only the G
    // entries it wrote itself, and shares g_(l+1) through LDS
    for (int l = f.L - 2; l >= 0; --l) {
      const int wo = f.w[l + 1], wn = f.w[l + 2];
      for (int j = lane; j < wn; j += 64) vstore(za, j, vload<T, C>(grow, f.goff[l + 1] + j));
      wave_sync();
      const T *Wn = P + int64_t(cs) * (f.poff[l + 1] + wn);   // W_(l+1) [wn][wo]
      for (int r = 0; r < kFfR; ++r) {
        const int k = lane + 64 * r;
        if (k >= wo) break;
        const V<T, C> acc = ff_dot<T, C>(vmake<T, C>(T(0), T(0)), Wn, wo, k, za, wn);
        vstore(grow, f.goff[l] + k, vmul(vload<T, C>(grow, f.goff[l] + k), acc));
      }
      wave_sync();
    }
  }
}

// the direction's weights transposed into the table layout (compute precision)
template <typename T, bool C>
__global__ void k_ff_prep_dir(FfDev f, const double *__restrict__ v, T *__restrict__ Vt,
                              const int *skip) {
  if (skip && *skip) return;
  for (int l = 0; l < f.L; ++l) {
    const int wi = f.w[l], wo = f.w[l + 1];
    const int64_t tot = int64_t(wi) * wo;
    for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < tot;
         e += int64_t(gridDim.x) * blockDim.x) {
      const int64_t k = e / wo, j = e % wo;
      vstore(Vt, f.toff[l] + e, vload<T, C>(v, f.poff[l] + wo + j * wi + k));
    }
  }
}

// y_s = (O v)_s; partial sums of y per block (fixed order)
template <typename T, bool C>
__global__ __launch_bounds__(256) void k_ff_jvp(FfDev f, FfWave fw, const int8_t *sigma,
                                                int64_t n, const T *Z, const T *G,
                                                const T *Vt, const double *v, double *y,
                                                double *ysum, const int *skip) {
  if (skip && *skip) return;
  constexpr int cs = C ? 2 : 1;
  __shared__ double part[4][2];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int8_t *sig;
  T *za, *zb;
  ff_wave_ptrs<T, C>(fw, wid, &sig, &za, &zb);
  (void)zb;
  const int64_t waves = int64_t(gridDim.x) * (blockDim.x >> 6);
  double br = 0.0, bi = 0.0;
  for (int64_t s = int64_t(blockIdx.x) * (blockDim.x >> 6) + wid; s < n; s += waves) {
    const T *zrow = Z + int64_t(cs) * s * f.zcols;
    const T *grow = G + int64_t(cs) * s * f.gcols;
    double tr = 0.0, ti = 0.0;
    for (int l = 0; l < f.L; ++l) {
      const int wi = f.w[l], wo = f.w[l + 1];
      if (l == 0)
        for (int i = lane; i < wi; i += 64) vstore(za, i, vmake<T, C>(T(sigma[s * f.N + i]), T(0)));
      else
        for (int i = lane; i < wi; i += 64) vstore(za, i, vload<T, C>(zrow, f.zoff[l] + i));
      wave_sync();
      const T *Vl = Vt + int64_t(cs) * f.toff[l];
      for (int r = 0; r < kFfR; ++r) {
        const int j = lane + 64 * r;
        if (j >= wo) break;
        const V<T, C> t = ff_dot<T, C>(vload<T, C>(v, f.poff[l] + j), Vl, wo, j, za, wi);
        const V<T, C> q = vmul(vload<T, C>(grow, f.goff[l] + j), t);
        tr += double(q.re);
        ti += double(q.im);
      }
      wave_sync();
    }
    tr = wave_sum(tr);
    ti = C ? wave_sum(ti) : 0.0;
    if (lane == 0) vstore(y, s, vmake<double, C>(tr, ti));
    br += tr;
    bi += ti;
  }
  if (ysum) {
    if (lane == 0) {
      part[wid][0] = br;
      part[wid][1] = bi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double a = 0.0, b = 0.0;
      for (int q = 0; q < int(blockDim.x >> 6); ++q) {
        a += part[q][0];
        b += part[q][1];
      }
      ysum[2 * blockIdx.x] = a;
      ysum[2 * blockIdx.x + 1] = b;
    }
  }
}

// O^dagger u for layer l: 64 x 64 tiles of (j, k), k = w[l] being the bias column,
// over the samples of split blockIdx.z; partials [split][j][k] in the compute precision
template <typename T, bool C>
__global__ __launch_bounds__(256) void k_ff_vjp(FfDev f, int l, const int8_t *sigma,
                                                int64_t n, int64_t per_split, const T *Z,
                                                const T *G, const double *u, T *part,
                                                const int *skip) {
  if (skip && *skip) return;
  constexpr int cs = C ? 2 : 1;
  __shared__ V<T, C> ga[16][64];
  __shared__ V<T, C> zb[16][64];
  const int wi = f.w[l], wo = f.w[l + 1], kc = wi + 1;
  const int j0 = blockIdx.x * 64, k0 = blockIdx.y * 64;
  const int64_t s_begin = int64_t(blockIdx.z) * per_split;
  const int64_t s_end = s_begin + per_split < n ? s_begin + per_split : n;
  const int tj = threadIdx.x >> 4, tk = threadIdx.x & 15;
  V<T, C> acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = vmake<T, C>(T(0), T(0));
  for (int64_t s0 = s_begin; s0 < s_end; s0 += 16) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = threadIdx.x + 256 * q;
      const int ss = e >> 6, jj = e & 63;
      const int64_t s = s0 + ss;
      V<T, C> gv = vmake<T, C>(T(0), T(0)), zv = vmake<T, C>(T(0), T(0));
      if (s < s_end) {
        const int j = j0 + jj, k = k0 + jj;
        if (j < wo) {
          const V<T, C> g = vload<T, C>(G + int64_t(cs) * s * f.gcols, f.goff[l] + j);
          const V<T, C> us = vload<T, C>(u, s);
          gv = vmul(vconj(g), us);
        }
        if (k < wi) {
          zv = l == 0 ? vmake<T, C>(T(sigma[s * f.N + k]), T(0))
                      : vconj(vload<T, C>(Z + int64_t(cs) * s * f.zcols, f.zoff[l] + k));
        } else if (k == wi) {
          zv = vmake<T, C>(T(1), T(0));
        }
      }
      ga[ss][jj] = gv;
      zb[ss][jj] = zv;
    }
    __syncthreads();
#pragma unroll 4
    for (int ss = 0; ss < 16; ++ss) {
      V<T, C> av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = ga[ss][tj * 4 + a];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = zb[ss][tk * 4 + b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = vadd(acc[a][b], vmul(av[a], bv[b]));
    }
    __syncthreads();
  }
  T *pp = part + int64_t(cs) * blockIdx.z * int64_t(wo) * kc;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int j = j0 + tj * 4 + a;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int k = k0 + tk * 4 + b;
      if (j < wo && k < kc) vstore(pp, int64_t(j) * kc + k, acc[a][b]);
    }
  }
}

// sum of the split partials of layer l (fixed order) into the params layout
template <typename T, bool C>
__global__ void k_ff_vjp_reduce(FfDev f, int l, int splits, const T *part, double *out,
                                const int *skip) {
  if (skip && *skip) return;
  const int wi = f.w[l], wo = f.w[l + 1], kc = wi + 1;
  const int64_t tot = int64_t(wo) * kc;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < tot;
       e += int64_t(gridDim.x) * blockDim.x) {
    V<double, C> acc = vmake<double, C>(0.0, 0.0);
    for (int q = 0; q < splits; ++q) acc = vadd(acc, vload<double, C>(part, q * tot + e));
    const int64_t j = e / kc, k = e % kc;
    const int64_t idx = k == wi ? f.poff[l] + j : f.poff[l] + wo + j * wi + k;
    vstore(out, idx, acc);
  }
}

FfWave ff_wave(const nqs_model *m) {
  FfWave fw;
  fw.Npad = (m->N + 15) / 16 * 16;
  const int el = (use_double(m) ? 8 : 4) * (m->is_complex ? 2 : 1);
  fw.zbytes = (m->ff.maxw * el + 15) / 16 * 16;
  return fw;
}

// wavefronts per block: 4, fewer when their LDS exceeds what a block may use
int ff_wpb(const nqs_model *m) {
  const int per = ff_wave(m).bytes();
  int w = 4;
  while (w > 1 && w * per > m->max_lds) --w;
  return w;
}

// LDS bytes of the staged weights of layers 1.. (0: not staged, the table is read from
// global memory): staged when they fit next to the wavefronts' buffers
size_t ff_stage_bytes(const nqs_model *m) {
  const FfDev &f = m->ff;
  if (f.L < 2) return 0;
  const size_t el = (use_double(m) ? 8 : 4) * (m->is_complex ? 2 : 1);
  const size_t b = size_t(f.tab - f.toff[1]) * el;
  return size_t(ff_wpb(m)) * ff_wave(m).bytes() + b <= size_t(m->max_lds) ? b : 0;
}

// dynamic LDS above 64 KiB, opted into once per kernel
hipError_t ff_lds_optin(const void *fn, size_t bytes, const nqs_model *m) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, m->max_lds);
}

unsigned ff_grid(const nqs_model *m, int64_t items) {
  const int wpb = ff_wpb(m);
  const int64_t b = cdiv(items, wpb);
  const int64_t cap = int64_t(m->cu_count) * 64;
  return unsigned(b < cap ? (b > 0 ? b : 1) : cap);
}

struct FfScratch {
  void *Z, *G, *Vt, *part;
  int64_t splits[kFfMaxLayers], per_split[kFfMaxLayers];
  size_t total;
};

FfScratch ff_scratch(const nqs_model *m, int64_t n, void *base) {
  const FfDev &f = m->ff;
  const size_t el = (use_double(m) ? 8 : 4) * (m->is_complex ? 2 : 1);
  FfScratch s;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += (bytes + 255) / 256 * 256;
    return (void *)((char *)base + o);
  };
  s.Z = take(size_t(n) * (f.zcols > 0 ? f.zcols : 1) * el);
  s.G = take(size_t(n) * f.gcols * el);
  s.Vt = take(size_t(f.tab) * el);
  size_t pmax = 0;
  for (int l = 0; l < f.L; ++l) {
    const int64_t tiles = cdiv(f.w[l + 1], 64) * cdiv(f.w[l] + 1, 64);
    int64_t sp = cdiv(int64_t(m->cu_count) * 8, tiles);
    const int64_t maxsp = cdiv(n, 64);
    sp = sp < 1 ? 1 : (sp > maxsp ? maxsp : sp);
    const int64_t per = cdiv(cdiv(n, sp), 16) * 16;
    s.per_split[l] = per;
    s.splits[l] = cdiv(n, per);
    const size_t b = size_t(s.splits[l]) * f.w[l + 1] * (f.w[l] + 1) * el;
    pmax = b > pmax ? b : pmax;
  }
  s.part = take(pmax);
  s.total = off;
  return s;
}

template <typename T, bool C>
hipError_t ff_launch_all(const nqs_model *m, int what, const void *params, const int8_t *sigma,
                         int64_t n, void *out, hipStream_t st) {
  const FfDev &f = m->ff;
  const FfWave fw = ff_wave(m);
  const int wpb = ff_wpb(m);
  const size_t lds = size_t(wpb) * fw.bytes();
  const T *P = (const T *)params;
  const T *Wt = (const T *)m->d_fftab;
  if (what == 0)
    hipLaunchKernelGGL((k_ff_log_psi<T, C>), dim3(ff_grid(m, n)), dim3(64 * wpb), lds, st, f,
                       fw, P, Wt, sigma, n, (double *)out);
  else {
    const size_t sb = ff_stage_bytes(m);
    if (sb) {
      const hipError_t e =
          ff_lds_optin(reinterpret_cast<const void *>(k_ff_eloc<T, C, true>), lds + sb, m);
      if (e != hipSuccess) return e;
      // as many blocks as stay resident, two per compute unit at most (the registers of
      // k_ff_eloc allow two wavefronts per SIMD); each stages the weights once
      const int64_t per_cu = int64_t(m->max_lds) / int64_t(lds + sb);
      const int64_t cap = int64_t(m->cu_count) * (per_cu < 1 ? 1 : (per_cu > 2 ? 2 : per_cu));
      const int64_t nb = cdiv(n, wpb);
      hipLaunchKernelGGL((k_ff_eloc<T, C, true>), dim3(unsigned(nb < cap ? nb : cap)),
                         dim3(64 * wpb), lds + sb, st, f, fw, dev_model(m), P, Wt, sigma, n,
                         (double *)out);
    } else {
      hipLaunchKernelGGL((k_ff_eloc<T, C, false>), dim3(ff_grid(m, n)), dim3(64 * wpb), lds, st,
                         f, fw, dev_model(m), P, Wt, sigma, n, (double *)out);
    }
  }
  return hipGetLastError();
}

#define NQS_FF_DISPATCH(FN, ...)                                                         \
  (use_double(m) ? (m->is_complex ? FN<double, true>(__VA_ARGS__)                      \
                                  : FN<double, false>(__VA_ARGS__))                    \
                 : (m->is_complex ? FN<float, true>(__VA_ARGS__)                       \
                                  : FN<float, false>(__VA_ARGS__)))

template <typename T, bool C>
hipError_t ff_tables_t(const nqs_model *m, const void *params, hipStream_t st) {
  const int64_t b = cdiv(m->ff.tab, 256);
  hipLaunchKernelGGL((k_ff_tables<T, C>), dim3(unsigned(b < 4096 ? b : 4096)), dim3(256), 0, st,
                     m->ff, (const T *)params, (T *)m->d_fftab);
  return hipGetLastError();
}

template <typename T, bool C>
hipError_t ff_sweep_t(const nqs_model *m, const void *params, int8_t *cs, int n_chains,
                      int n_sweeps, int n_discard, uint64_t seed, uint64_t counter,
                      int chain_offset, int8_t *samples, int64_t *n_acc, hipStream_t st) {
  FfSweepArgs a;
  a.chain_sigma = cs;
  a.n_chains = n_chains;
  a.n_sweeps = n_sweeps;
  a.n_discard = n_discard;
  a.k0 = uint32_t(seed & 0xffffffffu);
  a.k1 = uint32_t(seed >> 32);
  a.counter = uint32_t(counter);
  a.chain_offset = uint32_t(chain_offset);
  a.samples = samples;
  a.n_acc = n_acc;
  const FfWave fw = ff_wave(m);
  const int wpb = ff_wpb(m);
  const size_t sb = ff_stage_bytes(m);
  const size_t lds = size_t(wpb) * fw.bytes();
  if (sb) {
    const hipError_t e =
        ff_lds_optin(reinterpret_cast<const void *>(k_ff_sweep<T, C, true>), lds + sb, m);
    if (e != hipSuccess) return e;
  }
  time_begin(m, NQS_TIME_SWEEP);
  time_mark(m, NQS_TIME_SWEEP, 0, st);
  if (sb)
    hipLaunchKernelGGL((k_ff_sweep<T, C, true>), dim3(unsigned(cdiv(n_chains, wpb))),
                       dim3(64 * wpb), lds + sb, st, m->ff, fw, dev_model(m), (const T *)params,
                       (const T *)m->d_fftab, a);
  else
    hipLaunchKernelGGL((k_ff_sweep<T, C, false>), dim3(unsigned(cdiv(n_chains, wpb))),
                       dim3(64 * wpb), lds, st, m->ff, fw, dev_model(m), (const T *)params,
                       (const T *)m->d_fftab, a);
  time_mark(m, NQS_TIME_SWEEP, 1, st);
  return hipGetLastError();
}

template <typename T, bool C>
hipError_t ff_fb_t(const nqs_model *m, const void *params, const int8_t *sigma, int64_t n,
                   void *scratch, hipStream_t st) {
  const FfScratch s = ff_scratch(m, n, scratch);
  const FfWave fw = ff_wave(m);
  const int wpb = ff_wpb(m);
  hipLaunchKernelGGL((k_ff_fb<T, C>), dim3(ff_grid(m, n)), dim3(64 * wpb),
                     size_t(wpb) * fw.bytes(), st, m->ff, fw, (const T *)params,
                     (const T *)m->d_fftab, sigma, n, (T *)s.Z, (T *)s.G);
  return hipGetLastError();
}

template <typename T, bool C>
hipError_t ff_jvp_t(const nqs_model *m, const int8_t *sigma, int64_t n, const double *v,
                    void *scratch, double *y, double *ysum, const int *skip, hipStream_t st) {
  const FfScratch s = ff_scratch(m, n, scratch);
  const FfWave fw = ff_wave(m);
  const int wpb = ff_wpb(m);
  const int64_t b = cdiv(m->ff.tab, 256);
  time_mark(m, NQS_TIME_SV, 0, st);
  hipLaunchKernelGGL((k_ff_prep_dir<T, C>), dim3(unsigned(b < 4096 ? b : 4096)), dim3(256), 0,
                     st, m->ff, v, (T *)s.Vt, skip);
  hipLaunchKernelGGL((k_ff_jvp<T, C>), dim3(ff_grid(m, n)), dim3(64 * wpb),
                     size_t(wpb) * fw.bytes(), st, m->ff, fw, sigma, n, (const T *)s.Z,
                     (const T *)s.G, (const T *)s.Vt, v, y, ysum, skip);
  time_mark(m, NQS_TIME_SV, 1, st);
  return hipGetLastError();
}

template <typename T, bool C>
hipError_t ff_vjp_t(const nqs_model *m, const int8_t *sigma, int64_t n, const double *u,
                    void *scratch, double *out, const int *skip, hipStream_t st) {
  const FfScratch s = ff_scratch(m, n, scratch);
  const FfDev &f = m->ff;
  time_mark(m, NQS_TIME_SV, 0, st);
  for (int l = 0; l < f.L; ++l) {
    const dim3 grid(unsigned(cdiv(f.w[l + 1], 64)), unsigned(cdiv(f.w[l] + 1, 64)),
                    unsigned(s.splits[l]));
    hipLaunchKernelGGL((k_ff_vjp<T, C>), grid, dim3(256), 0, st, f, l, sigma, n,
                       s.per_split[l], (const T *)s.Z, (const T *)s.G, u, (T *)s.part, skip);
    const int64_t tot = int64_t(f.w[l + 1]) * (f.w[l] + 1);
    const int64_t b = cdiv(tot, 256);
    hipLaunchKernelGGL((k_ff_vjp_reduce<T, C>), dim3(unsigned(b < 4096 ? b : 4096)), dim3(256),
                       0, st, f, l, int(s.splits[l]), (const T *)s.part, out, skip);
  }
  time_mark(m, NQS_TIME_SV, 1, st);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_ff_tables(const nqs_model *m, const void *params, hipStream_t st) {
  return NQS_FF_DISPATCH(ff_tables_t, m, params, st);
}

hipError_t launch_ff_log_psi(const nqs_model *m, const void *params, const int8_t *sigma,
                             int64_t n, void *out, hipStream_t st) {
  return NQS_FF_DISPATCH(ff_launch_all, m, 0, params, sigma, n, out, st);
}

hipError_t launch_ff_local_energy(const nqs_model *m, const void *params, const int8_t *sigma,
                                  int64_t n, void *eloc, hipStream_t st) {
  time_begin(m, NQS_TIME_ELOC);
  time_mark(m, NQS_TIME_ELOC, 0, st);
  hipError_t e = NQS_FF_DISPATCH(ff_launch_all, m, 1, params, sigma, n, eloc, st);
  time_mark(m, NQS_TIME_ELOC, 1, st);
  return e;
}

hipError_t launch_ff_sweep(const nqs_model *m, const void *params, int8_t *chain_sigma,
                           int n_chains, int n_sweeps, int n_discard, uint64_t seed,
                           uint64_t counter, int chain_offset, int8_t *samples, int64_t *n_acc,
                           hipStream_t st) {
  return NQS_FF_DISPATCH(ff_sweep_t, m, params, chain_sigma, n_chains, n_sweeps, n_discard,
                         seed, counter, chain_offset, samples, n_acc, st);
}

size_t ff_grad_scratch_bytes(const nqs_model *m, int64_t n) {
  return ff_scratch(m, n, nullptr).total;
}

hipError_t launch_ff_fb(const nqs_model *m, const void *params, const int8_t *sigma, int64_t n,
                        void *scratch, hipStream_t st) {
  return NQS_FF_DISPATCH(ff_fb_t, m, params, sigma, n, scratch, st);
}

int64_t ff_jvp_blocks(const nqs_model *m, int64_t n) { return ff_grid(m, n); }

hipError_t launch_ff_jvp(const nqs_model *m, const void *params, const int8_t *sigma,
                         int64_t n, const double *v, void *scratch, double *y, double *ysum,
                         const int *skip, hipStream_t st) {
  (void)params;
  return NQS_FF_DISPATCH(ff_jvp_t, m, sigma, n, v, scratch, y, ysum, skip, st);
}

hipError_t launch_ff_vjp(const nqs_model *m, const int8_t *sigma, int64_t n, const double *u,
                         void *scratch, double *out, const int *skip, hipStream_t st) {
  return NQS_FF_DISPATCH(ff_vjp_t, m, sigma, n, u, scratch, out, skip, st);
}
