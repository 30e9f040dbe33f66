// Parameter tables, chain initialisation, Metropolis sweeps, local energies and log psi.
//
// RBM (Sec. 2.2.2): log psi(s) = sum_i a_i s_i + sum_j ln cosh theta_j,
// theta_j = b_j + sum_i W_ji s_i. Moving from s to s' changes theta by delta_j, and
//   psi(s')/psi(s) = exp(sum_i a_i (s'_i - s_i)) * prod_j cosh(theta_j + delta_j)/cosh(theta_j)
//                  = exp(...) * prod_j [cosh(delta_j) + tanh(theta_j) sinh(delta_j)].
// A flip of site i (spin s) has delta_j = -2 s W_ji; an exchange on bond (i, k) with
// s_k = -s has delta_j = -2 s (W_ji - W_jk). cosh/sinh of 2 W_ji and of 2 (W_ji - W_jk)
// do not depend on the configuration, so they are tabulated once per call and each ratio
// term costs one complex multiply-add, with no transcendental function.
#include "internal.hpp"

namespace {

__device__ __forceinline__ float bf16_round(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xffff0000u);
}

// ---------------------------------------------------------------------------------
// Tables: one thread per element of the three index ranges
//   [0, N*M)            W transposed + flip tables
//   [N*M, N*M+Btot*M)   bond tables
//   then M + N + Btot   bias, a, a-factors
// ---------------------------------------------------------------------------------
template <typename T, bool C, typename PT>
__global__ void k_tables(DevModel dm, Tables<T> tb, const PT *__restrict__ p, int quant,
                         int need_flip, int need_bond) {
  const int N = dm.N, M = dm.M, B = dm.Btot;
  const int64_t nW = int64_t(N) * M, nB = int64_t(B) * M;
  const int64_t total = nW + nB + M + N + B;
  const int64_t offW = N + M;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    if (e < nW) {
      int i = int(e / M), j = int(e % M);
      V<double, C> w = vload<double, C>(p, offW + int64_t(j) * N + i);
      if (quant) {
        w.re = bf16_round(float(w.re));
        if (C) w.im = bf16_round(float(w.im));
      }
      vstore<T, C>(tb.Wt, int64_t(i) * M + j, vcast<double, C, T>(w));
      if (need_flip) {
        double x = 2 * w.re, y = 2 * w.im;
        double ch = cosh(x), sh = sinh(x), sy = 0, cy = 1;
        if (C) sincos(y, &sy, &cy);
        V<double, C> cc = vmake<double, C>(ch * cy, sh * sy);
        V<double, C> ss = vmake<double, C>(sh * cy, ch * sy);
        vstore<T, C>(tb.fC, int64_t(i) * M + j, vcast<double, C, T>(cc));
        vstore<T, C>(tb.fS, int64_t(i) * M + j, vcast<double, C, T>(ss));
        vstore<T, C>(tb.fCt, int64_t(j) * N + i, vcast<double, C, T>(cc));
        vstore<T, C>(tb.fSt, int64_t(j) * N + i, vcast<double, C, T>(ss));
      }
    } else if (e < nW + nB) {
      if (!need_bond) continue;
      int64_t q = e - nW;
      int b = int(q / M), j = int(q % M);
      int i = dm.bonds[2 * b], k = dm.bonds[2 * b + 1];
      V<double, C> wi = vload<double, C>(p, offW + int64_t(j) * N + i);
      V<double, C> wk = vload<double, C>(p, offW + int64_t(j) * N + k);
      if (quant) {
        wi.re = bf16_round(float(wi.re));
        wk.re = bf16_round(float(wk.re));
        if (C) {
          wi.im = bf16_round(float(wi.im));
          wk.im = bf16_round(float(wk.im));
        }
      }
      double x = 2 * (wi.re - wk.re), y = C ? 2 * (wi.im - wk.im) : 0.0;
      double ch = cosh(x), sh = sinh(x), sy = 0, cy = 1;
      if (C) sincos(y, &sy, &cy);
      V<double, C> cc = vmake<double, C>(ch * cy, sh * sy);
      V<double, C> ss = vmake<double, C>(sh * cy, ch * sy);
      vstore<T, C>(tb.bC, int64_t(b) * M + j, vcast<double, C, T>(cc));
      vstore<T, C>(tb.bS, int64_t(b) * M + j, vcast<double, C, T>(ss));
      vstore<T, C>(tb.bCt, int64_t(j) * B + b, vcast<double, C, T>(cc));
      vstore<T, C>(tb.bSt, int64_t(j) * B + b, vcast<double, C, T>(ss));
      if (tb.Wd && b < dm.B0) vstore<T, C>(tb.Wd, int64_t(b) * M + j, vcast<double, C, T>(vsub(wi, wk)));
    } else {
      int64_t q = e - nW - nB;
      if (q < M) {
        vstore<T, C>(tb.bv, q, vcast<double, C, T>(vload<double, C>(p, N + q)));
      } else if (q < M + N) {
        int i = int(q - M);
        V<double, C> a = vload<double, C>(p, i);
        tb.av[2 * i] = a.re;
        tb.av[2 * i + 1] = C ? a.im : 0.0;
        // exp(-2 s a_i): s = +1 -> row 0, s = -1 -> row 1
        for (int r = 0; r < 2; ++r) {
          double sgn = r == 0 ? -2.0 : 2.0;
          double mag = exp(sgn * a.re), sy = 0, cy = 1;
          if (C) sincos(sgn * a.im, &sy, &cy);
          tb.fa[2 * (int64_t(r) * N + i)] = mag * cy;
          tb.fa[2 * (int64_t(r) * N + i) + 1] = mag * sy;
        }
      } else {
        int b = int(q - M - N);
        int i = dm.bonds[2 * b], k = dm.bonds[2 * b + 1];
        V<double, C> ai = vload<double, C>(p, i), ak = vload<double, C>(p, k);
        double dr = ai.re - ak.re, di = C ? ai.im - ak.im : 0.0;
        for (int r = 0; r < 2; ++r) {
          double sgn = r == 0 ? -2.0 : 2.0;
          double mag = exp(sgn * dr), sy = 0, cy = 1;
          if (C) sincos(sgn * di, &sy, &cy);
          tb.ba[2 * (int64_t(r) * B + b)] = mag * cy;
          tb.ba[2 * (int64_t(r) * B + b) + 1] = mag * sy;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------------
// Chain initialisation: Philox4x32-10, counter (chain, 0, site, TAG_INIT).
// ---------------------------------------------------------------------------------
__global__ void k_init_flip(int8_t *sig, int n_chains, int N, uint32_t k0, uint32_t k1,
                            uint32_t chain_offset) {
  int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (e >= int64_t(n_chains) * N) return;
  int c = int(e / N), i = int(e % N);
  Philox4 w = philox4x32_10(chain_offset + uint32_t(c), 0u, uint32_t(i), TAG_INIT, k0, k1);
  sig[e] = (w.w[0] >> 31) == 0 ? int8_t(1) : int8_t(-1);
}

// zero magnetisation: N/2 up then N/2 down, shuffled by Fisher-Yates from the last site
__global__ void k_init_sz0(int8_t *sig, int n_chains, int N, uint32_t k0, uint32_t k1,
                           uint32_t chain_offset) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_chains) return;
  int8_t *row = sig + int64_t(c) * N;
  for (int i = 0; i < N; ++i) row[i] = i < N / 2 ? int8_t(1) : int8_t(-1);
  for (int k = N - 1; k >= 1; --k) {
    Philox4 w = philox4x32_10(chain_offset + uint32_t(c), 0u, uint32_t(k), TAG_INIT, k0, k1);
    int r = rng_index(w.w[0], uint32_t(k + 1));
    int8_t t = row[k];
    row[k] = row[r];
    row[r] = t;
  }
}

// ---------------------------------------------------------------------------------
// Local energy of one configuration (Eq. 5), evaluated by one wavefront: sig (LDS, N
// spins) and tj (LDS, tanh theta_j) are given. Each lane takes connected configurations
// (a flipped site for TFIM, an anti-aligned bond for Heisenberg) and multiplies their M
// ratio terms serially from the hidden-major tables (contiguous across lanes). Returns
// the wave-uniform (re, im) in double.
// ---------------------------------------------------------------------------------
template <typename T, bool C>
__device__ __forceinline__ void eloc_wave(const DevModel &dm, const Tables<T> &tb,
                                          const int8_t *sig, const V<T, C> *tj, int lane,
                                          double &out_re, double &out_im) {
  const int N = dm.N, M = dm.M, B = dm.Btot;
  double diag = 0.0;
  for (int b = lane; b < B; b += 64)
    diag += dm.bond_diag[b] * double(sig[dm.bonds[2 * b]]) * double(sig[dm.bonds[2 * b + 1]]);
  double er = 0.0, ei = 0.0;
  const bool tfim = dm.ham == NQS_TFIM;
  const int ncand = tfim ? (dm.h != 0.0 ? N : 0) : B;
  const int stride = tfim ? N : B;
  const T *Ct = tfim ? tb.fCt : tb.bCt;
  const T *St = tfim ? tb.fSt : tb.bSt;
  for (int c = lane; c < ncand; c += 64) {
    int s;
    double el;
    const double *af;
    if (tfim) {
      s = sig[c];
      el = -dm.h;
      af = tb.fa + 2 * (int64_t(s > 0 ? 0 : 1) * N + c);
    } else {
      const int i = dm.bonds[2 * c], k = dm.bonds[2 * c + 1];
      s = sig[i];
      el = dm.bond_off[c];
      if (sig[k] == s || el == 0.0) continue;
      af = tb.ba + 2 * (int64_t(s > 0 ? 0 : 1) * B + c);
    }
    const T ts = T(s);
    V<T, C> p = vmake<T, C>(T(1), T(0));
    int pe = 0;
    for (int j = 0; j < M; ++j) {
      V<T, C> cc = vload<T, C>(Ct, int64_t(j) * stride + c);
      V<T, C> ss = vload<T, C>(St, int64_t(j) * stride + c);
      p = vmul(p, vsub(cc, vscale(vmul(tj[j], ss), ts)));
      if ((j & 3) == 3) vrenorm(p, pe);
    }
    vrenorm(p, pe);
    const double rr = ldexp(double(p.re), pe), ri = C ? ldexp(double(p.im), pe) : 0.0;
    er += el * (rr * af[0] - ri * af[1]);
    ei += el * (rr * af[1] + ri * af[0]);
  }
  out_re = wave_sum_dpp(diag) + wave_sum_dpp(er);
  out_im = C ? wave_sum_dpp(ei) : 0.0;
}

// ---------------------------------------------------------------------------------
// Metropolis sweeps. One chain per wavefront; lane l owns hidden units l + 64 r (r < R):
// theta_j cached in double (exact running sums of +/-2 W), t_j = tanh(theta_j) in T.
// A proposal costs R ratio terms per lane (C - s t S), a DPP product reduction carried as
// mantissa x 2^exponent, and a wave-uniform accept decision in double. On acceptance
// theta moves by -2 s W_row and t by the addition formula t' = (C t - s S) / term, whose
// denominator is the ratio term already computed; t is recomputed from theta at the end
// of every sweep, so rounding does not accumulate over sweeps. Spins live in LDS; the
// move tables (C, S, W rows) are staged in LDS when they fit (TL), and the rows of the
// next proposal are fetched one step ahead (the counter-based stream makes it known).
// After each recorded sweep the chain's local energy is evaluated from its cached t.
// ---------------------------------------------------------------------------------
struct SweepArgs {
  int8_t *chain_sigma;
  int n_chains, n_sweeps, n_discard;
  uint32_t k0, k1, counter, chain_offset;
  int8_t *samples;
  int64_t *n_acc;
  double *eloc;
  int tab_rows;      // rows of the move tables (N for flips, B0 for exchanges)
  int wave_bytes;    // per-wavefront LDS: t (M values) then spins
};

template <typename T, bool C, int R, bool TL>
__global__ __launch_bounds__(256) void k_sweep(DevModel dm, Tables<T> tb, SweepArgs a) {
  extern __shared__ __align__(16) unsigned char lds_u8[];
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int chain = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + wid);
  const int N = dm.N, M = dm.M;
  const int cs = C ? 2 : 1;
  const bool flip = dm.move == NQS_MOVE_FLIP;
  const int rows = a.tab_rows;
  const T *gC = flip ? tb.fC : tb.bC;
  const T *gS = flip ? tb.fS : tb.bS;
  const T *gW = flip ? tb.Wt : tb.Wd;
  T *lC = reinterpret_cast<T *>(lds_u8);
  T *lS = lC + int64_t(rows) * M * cs;
  T *lW = lS + int64_t(rows) * M * cs;
  const int64_t tab_bytes = TL ? int64_t(3) * rows * M * cs * int64_t(sizeof(T)) : 0;
  if constexpr (TL) {
    const int64_t cnt = int64_t(rows) * M * cs;
    for (int64_t e = threadIdx.x; e < cnt; e += blockDim.x) {
      lC[e] = gC[e];
      lS[e] = gS[e];
      lW[e] = gW[e];
    }
    __syncthreads();
  }
  if (chain >= a.n_chains) return;
  unsigned char *wbase = lds_u8 + tab_bytes + int64_t(wid) * a.wave_bytes;
  V<T, C> *tj = reinterpret_cast<V<T, C> *>(wbase);
  int8_t *sig = reinterpret_cast<int8_t *>(wbase + ((M * int(sizeof(V<T, C>)) + 15) / 16) * 16);
  for (int i = lane; i < N; i += 64) sig[i] = a.chain_sigma[int64_t(chain) * N + i];
  wave_sync();

  auto row_ld = [&](const T *lp, const T *gp, int row, int j) -> V<T, C> {
    if constexpr (TL)
      return vload<T, C>(lp, int64_t(row) * M + j);
    else
      return vload<T, C>(gp, int64_t(row) * M + j);
  };

  double thr[R], thi[R];
  V<T, C> t[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int j = lane + 64 * r;
    thr[r] = 0.0;
    thi[r] = 0.0;
    t[r] = vmake<T, C>(T(0), T(0));
    if (j < M) {
      V<double, C> acc = vload<double, C>(tb.bv, j);
      for (int i = 0; i < N; ++i) {
        const double s = double(sig[i]);
        V<double, C> w = vload<double, C>(tb.Wt, int64_t(i) * M + j);
        acc.re += s * w.re;
        if (C) acc.im += s * w.im;
      }
      thr[r] = acc.re;
      thi[r] = C ? acc.im : 0.0;
      t[r] = vtanh<T, C>(vmake<T, C>(T(thr[r]), T(thi[r])));
    }
  }

  const uint32_t cid = a.chain_offset + uint32_t(chain);
  const int total = a.n_discard + a.n_sweeps;
  // proposal (sweep, step) -> random words, table row and the sites it touches
  auto propose = [&](int sw, int st, Philox4 &w, int &row, int &i, int &k) {
    w = philox4x32_10(cid, a.counter + uint32_t(sw), uint32_t(st), TAG_PROPOSAL, a.k0, a.k1);
    if (flip) {
      i = rng_index(w.w[0], uint32_t(N));
      row = i;
      k = i;
    } else {
      row = rng_index(w.w[0], uint32_t(dm.B0));
      i = dm.bonds[2 * row];
      k = dm.bonds[2 * row + 1];
    }
  };
  // with few hidden units per lane the next proposal's rows are fetched one step ahead;
  // with many, the R independent loads of a step already overlap
  constexpr bool PF = R <= 4;
  constexpr int RP = PF ? R : 1;
  Philox4 wc;
  int rowc = 0, ic = 0, kc = 0;
  V<T, C> cc[R], ss[R], ww[R];
  auto load_rows = [&](int row, V<T, C> *c_, V<T, C> *s_, V<T, C> *w_) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int j = lane + 64 * r < M ? lane + 64 * r : 0;
      c_[r] = row_ld(lC, gC, row, j);
      s_[r] = row_ld(lS, gS, row, j);
      w_[r] = row_ld(lW, gW, row, j);
    }
  };
  if constexpr (PF) {
    propose(0, 0, wc, rowc, ic, kc);
    load_rows(rowc, cc, ss, ww);
  }
  int64_t acc_count = 0;
  for (int sw = 0; sw < total; ++sw) {
    for (int st = 0; st < N; ++st) {
      Philox4 wn = wc;
      int rown = rowc, in_ = ic, kn = kc;
      V<T, C> nc[RP], ns[RP], nw[RP];
      if constexpr (PF) {
        int nsw = sw, nst = st + 1;
        if (nst == N) {
          nst = 0;
          ++nsw;
        }
        if (nsw < total) propose(nsw, nst, wn, rown, in_, kn);
        load_rows(rown, nc, ns, nw);
      } else {
        propose(sw, st, wc, rowc, ic, kc);
        load_rows(rowc, cc, ss, ww);
      }

      const int s = __builtin_amdgcn_readfirstlane(int(sig[ic]));
      const int sk = flip ? -s : __builtin_amdgcn_readfirstlane(int(sig[kc]));
      if (sk != s) {  // an exchange of equal spins is the identity move
        const T ts = T(s);
        V<T, C> term[R];
        T pm = T(1);
        int pe = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          term[r] = vsub(cc[r], vscale(vmul(t[r], ss[r]), ts));
          if (lane + 64 * r < M) pm *= vabs2(term[r]);
          if ((r & 3) == 3) {
            int e;
            pm = nfrexp(pm, &e);
            pe += e;
          }
        }
        {
          int e;
          pm = nfrexp(pm, &e);
          pe += e;
        }
        const T pmw = wave_prod_dpp(pm, pe);
        const double *af = flip ? tb.fa + 2 * (int64_t(s > 0 ? 0 : 1) * N + rowc)
                                : tb.ba + 2 * (int64_t(s > 0 ? 0 : 1) * dm.Btot + rowc);
        const double q = ldexp(double(pmw), pe) * (af[0] * af[0] + af[1] * af[1]);
        const double u = rng_uniform(wc.w[1], wc.w[2]);
        const int accept = __builtin_amdgcn_readfirstlane(int((q >= 1.0) || (u < q)));
        if (accept) {
#pragma unroll
          for (int r = 0; r < R; ++r) {
            if (lane + 64 * r < M) {
              thr[r] -= 2.0 * double(s) * double(ww[r].re);
              if (C) thi[r] -= 2.0 * double(s) * double(ww[r].im);
              t[r] = vdiv(vsub(vmul(cc[r], t[r]), vscale(ss[r], ts)), term[r]);
            }
          }
          if (lane == 0) {
            sig[ic] = int8_t(-s);
            if (!flip) sig[kc] = int8_t(s);
          }
          wave_sync();
          ++acc_count;
        }
      }
      if constexpr (PF) {
        wc = wn;
        rowc = rown;
        ic = in_;
        kc = kn;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          cc[r] = nc[r];
          ss[r] = ns[r];
          ww[r] = nw[r];
        }
      }
    }
    // end of sweep: tanh from the exact angles
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (lane + 64 * r < M) t[r] = vtanh<T, C>(vmake<T, C>(T(thr[r]), T(thi[r])));
    if (sw >= a.n_discard) {
      const int64_t smp = int64_t(sw - a.n_discard) * a.n_chains + chain;
      int8_t *dst = a.samples + smp * N;
      for (int i = lane; i < N; i += 64) dst[i] = sig[i];
      if (a.eloc) {
#pragma unroll
        for (int r = 0; r < R; ++r)
          if (lane + 64 * r < M) tj[lane + 64 * r] = t[r];
        wave_sync();
        double er, ei;
        eloc_wave<T, C>(dm, tb, sig, tj, lane, er, ei);
        if (lane == 0) {
          if (C) {
            a.eloc[2 * smp] = er;
            a.eloc[2 * smp + 1] = ei;
          } else {
            a.eloc[smp] = er;
          }
        }
        wave_sync();
      }
    }
  }
  for (int i = lane; i < N; i += 64) a.chain_sigma[int64_t(chain) * N + i] = sig[i];
  if (lane == 0 && a.n_acc) a.n_acc[chain] = acc_count;
}

// ---------------------------------------------------------------------------------
// Local energy of arbitrary configurations. One sample per wavefront: theta in double,
// tanh into LDS, then eloc_wave.
// ---------------------------------------------------------------------------------
template <typename T, bool C>
__global__ __launch_bounds__(256) void k_local_energy(DevModel dm, Tables<T> tb,
                                                       const int8_t *__restrict__ sigma,
                                                       int64_t n, double *eloc, int Npad,
                                                       int lds_wave_bytes) {
  extern __shared__ __align__(16) unsigned char lds_u8[];
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int64_t smp = int64_t(blockIdx.x) * (blockDim.x >> 6) + wid;
  if (smp >= n) return;
  const int N = dm.N, M = dm.M;
  unsigned char *base = lds_u8 + int64_t(wid) * lds_wave_bytes;
  int8_t *sig = reinterpret_cast<int8_t *>(base);
  V<T, C> *tj = reinterpret_cast<V<T, C> *>(base + Npad);
  for (int i = lane; i < N; i += 64) sig[i] = sigma[smp * N + i];
  wave_sync();
  for (int j = lane; j < M; j += 64) {
    V<double, C> acc = vload<double, C>(tb.bv, j);
    for (int i = 0; i < N; ++i) {
      double s = double(sig[i]);
      V<double, C> w = vload<double, C>(tb.Wt, int64_t(i) * M + j);
      acc.re += s * w.re;
      if (C) acc.im += s * w.im;
    }
    tj[j] = vtanh<T, C>(vmake<T, C>(T(acc.re), T(acc.im)));
  }
  wave_sync();
  double er, ei;
  eloc_wave<T, C>(dm, tb, sig, tj, lane, er, ei);
  if (lane == 0) {
    if (C) {
      eloc[2 * smp] = er;
      eloc[2 * smp + 1] = ei;
    } else {
      eloc[smp] = er;
    }
  }
}

// ---------------------------------------------------------------------------------
// log psi. One sample per wavefront; theta, ln cosh and the sums in double for every
// compute precision (near the complex zeros of cosh theta, rounding theta to FP32 alone
// would dominate the error; log psi is not on the sampling or SR path).
// ---------------------------------------------------------------------------------
template <typename T, bool C>
__global__ __launch_bounds__(256) void k_log_psi(DevModel dm, Tables<T> tb,
                                                  const int8_t *__restrict__ sigma, int64_t n,
                                                  double *out, int Npad) {
  extern __shared__ int8_t lds_s8[];
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int64_t smp = int64_t(blockIdx.x) * (blockDim.x >> 6) + wid;
  if (smp >= n) return;
  const int N = dm.N, M = dm.M;
  int8_t *sig = lds_s8 + wid * Npad;
  for (int i = lane; i < N; i += 64) sig[i] = sigma[smp * N + i];
  wave_sync();
  double lr = 0.0, li = 0.0;
  for (int j = lane; j < M; j += 64) {
    V<double, C> acc = vload<double, C>(tb.bv, j);
    for (int i = 0; i < N; ++i) {
      double s = double(sig[i]);
      V<double, C> w = vload<double, C>(tb.Wt, int64_t(i) * M + j);
      acc.re += s * w.re;
      if (C) acc.im += s * w.im;
    }
    V<double, C> lc = vlncosh<double, C>(acc);
    lr += lc.re;
    if (C) li += lc.im;
  }
  for (int i = lane; i < N; i += 64) {
    lr += tb.av[2 * i] * double(sig[i]);
    li += tb.av[2 * i + 1] * double(sig[i]);
  }
  lr = wave_sum(lr);
  li = wave_sum(li);
  if (lane == 0) {
    if (C) {
      out[2 * smp] = lr;
      out[2 * smp + 1] = li;
    } else {
      out[smp] = lr;
    }
  }
}

template <typename T>
Tables<T> tables_of(const nqs_model *m) {
  Tables<T> tb;
  tb.Wt = (T *)m->tab_ptrs[0];
  tb.bv = (T *)m->tab_ptrs[1];
  tb.fC = (T *)m->tab_ptrs[2];
  tb.fS = (T *)m->tab_ptrs[3];
  tb.bC = (T *)m->tab_ptrs[4];
  tb.bS = (T *)m->tab_ptrs[5];
  tb.fCt = (T *)m->tab_ptrs[6];
  tb.fSt = (T *)m->tab_ptrs[7];
  tb.bCt = (T *)m->tab_ptrs[8];
  tb.bSt = (T *)m->tab_ptrs[9];
  tb.fa = (double *)m->tab_ptrs[10];
  tb.ba = (double *)m->tab_ptrs[11];
  tb.av = (double *)m->tab_ptrs[12];
  tb.Wd = (T *)m->tab_ptrs[13];
  return tb;
}

inline int round_up(int x, int a) { return (x + a - 1) / a * a; }

template <typename T, bool C>
hipError_t tables_t(const nqs_model *m, const void *params, hipStream_t st) {
  DevModel dm = dev_model(m);
  Tables<T> tb = tables_of<T>(m);
  int64_t total = int64_t(m->N) * m->M + int64_t(m->Btot) * m->M + m->M + m->N + m->Btot;
  int blocks = int((total + 255) / 256);
  if (blocks > 65536) blocks = 65536;
  int quant = m->prec == NQS_BF16;
  if (m->prec == NQS_F64)
    hipLaunchKernelGGL((k_tables<T, C, double>), dim3(blocks), dim3(256), 0, st, dm, tb,
                       (const double *)params, quant, int(m->need_flip), int(m->need_bond));
  else
    hipLaunchKernelGGL((k_tables<T, C, float>), dim3(blocks), dim3(256), 0, st, dm, tb,
                       (const float *)params, quant, int(m->need_flip), int(m->need_bond));
  return hipGetLastError();
}

template <typename T, bool C, int R>
hipError_t sweep_r(const nqs_model *m, int8_t *cs, int n_chains, int n_sweeps, int n_discard,
                   uint64_t seed, uint64_t counter, int chain_offset, int8_t *samples,
                   int64_t *n_acc, void *eloc, hipStream_t st) {
  const int wpb = 4;
  SweepArgs a;
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
  a.eloc = (double *)eloc;
  a.tab_rows = m->move == NQS_MOVE_FLIP ? m->N : m->B[0];
  a.wave_bytes = round_up(m->M * int(sizeof(V<T, C>)), 16) + round_up(m->N, 16);
  const size_t wave_lds = size_t(wpb) * a.wave_bytes;
  const size_t tab_lds = size_t(3) * a.tab_rows * m->M * sizeof(T) * (C ? 2 : 1);
  dim3 grid((n_chains + wpb - 1) / wpb);
  if (tab_lds + wave_lds <= size_t(m->max_lds)) {
    hipLaunchKernelGGL((k_sweep<T, C, R, true>), grid, dim3(64 * wpb), tab_lds + wave_lds, st,
                       dev_model(m), tables_of<T>(m), a);
  } else {
    hipLaunchKernelGGL((k_sweep<T, C, R, false>), grid, dim3(64 * wpb), wave_lds, st,
                       dev_model(m), tables_of<T>(m), a);
  }
  return hipGetLastError();
}

template <typename T, bool C>
hipError_t sweep_t(const nqs_model *m, int8_t *cs, int n_chains, int n_sweeps, int n_discard,
                   uint64_t seed, uint64_t counter, int chain_offset, int8_t *samples,
                   int64_t *n_acc, void *eloc, hipStream_t st) {
  int r = (m->M + 63) / 64;
#define NQS_SWEEP_CASE(RR)                                                                 \
  if (r <= RR)                                                                             \
    return sweep_r<T, C, RR>(m, cs, n_chains, n_sweeps, n_discard, seed, counter,          \
                             chain_offset, samples, n_acc, eloc, st);
  NQS_SWEEP_CASE(1)
  NQS_SWEEP_CASE(2)
  NQS_SWEEP_CASE(4)
  NQS_SWEEP_CASE(8)
  NQS_SWEEP_CASE(16)
  NQS_SWEEP_CASE(32)
#undef NQS_SWEEP_CASE
  return hipErrorInvalidValue;
}

template <typename T, bool C>
hipError_t eloc_t(const nqs_model *m, const int8_t *sigma, int64_t n, void *eloc,
                  hipStream_t st) {
  if (n == 0) return hipSuccess;
  int Npad = round_up(m->N, 16);
  int wave_bytes = Npad + round_up(m->M * int(sizeof(V<T, C>)), 16);
  int wpb = 4;
  while (wpb > 1 && wpb * wave_bytes > 64 * 1024) wpb /= 2;
  dim3 grid(unsigned((n + wpb - 1) / wpb));
  hipLaunchKernelGGL((k_local_energy<T, C>), grid, dim3(64 * wpb), size_t(wpb) * wave_bytes,
                     st, dev_model(m), tables_of<T>(m), sigma, n, (double *)eloc, Npad,
                     wave_bytes);
  return hipGetLastError();
}

template <typename T, bool C>
hipError_t logpsi_t(const nqs_model *m, const int8_t *sigma, int64_t n, void *out,
                    hipStream_t st) {
  if (n == 0) return hipSuccess;
  int Npad = round_up(m->N, 16);
  const int wpb = 4;
  dim3 grid(unsigned((n + wpb - 1) / wpb));
  hipLaunchKernelGGL((k_log_psi<T, C>), grid, dim3(64 * wpb), size_t(wpb) * Npad, st,
                     dev_model(m), tables_of<T>(m), sigma, n, (double *)out, Npad);
  return hipGetLastError();
}

}  // namespace

#define NQS_DISPATCH(FN, ...)                                                              \
  (use_double(m) ? (m->is_complex ? FN<double, true>(__VA_ARGS__)                          \
                                  : FN<double, false>(__VA_ARGS__))                        \
                 : (m->is_complex ? FN<float, true>(__VA_ARGS__)                           \
                                  : FN<float, false>(__VA_ARGS__)))

hipError_t launch_tables(const nqs_model *m, const void *params, hipStream_t st) {
  return NQS_DISPATCH(tables_t, m, params, st);
}

hipError_t launch_chain_init(const nqs_model *m, int8_t *sig, int n_chains, uint64_t seed,
                             int chain_offset, hipStream_t st) {
  uint32_t k0 = uint32_t(seed & 0xffffffffu), k1 = uint32_t(seed >> 32);
  if (m->move == NQS_MOVE_FLIP) {
    int64_t total = int64_t(n_chains) * m->N;
    hipLaunchKernelGGL(k_init_flip, dim3(unsigned((total + 255) / 256)), dim3(256), 0, st, sig,
                       n_chains, m->N, k0, k1, uint32_t(chain_offset));
  } else {
    hipLaunchKernelGGL(k_init_sz0, dim3(unsigned((n_chains + 63) / 64)), dim3(64), 0, st, sig,
                       n_chains, m->N, k0, k1, uint32_t(chain_offset));
  }
  return hipGetLastError();
}

hipError_t launch_sweep(const nqs_model *m, int8_t *chain_sigma, int n_chains, int n_sweeps,
                        int n_discard, uint64_t seed, uint64_t counter, int chain_offset,
                        int8_t *samples, int64_t *n_acc, void *eloc, hipStream_t st) {
  return NQS_DISPATCH(sweep_t, m, chain_sigma, n_chains, n_sweeps, n_discard, seed, counter,
                      chain_offset, samples, n_acc, eloc, st);
}

hipError_t launch_local_energy(const nqs_model *m, const int8_t *sigma, int64_t n, void *eloc,
                               hipStream_t st) {
  return NQS_DISPATCH(eloc_t, m, sigma, n, eloc, st);
}

hipError_t launch_log_psi(const nqs_model *m, const int8_t *sigma, int64_t n, void *out,
                          hipStream_t st) {
  return NQS_DISPATCH(logpsi_t, m, sigma, n, out, st);
}
