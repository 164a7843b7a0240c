// HIP kernels for gfx950: one time step of the 1D Maxwell-Bloch system per
// cell and lane.  State is structure-of-arrays (E, H and the M = N*N - 1
// density parameters as separate planes); per-material coefficients are
// read through the constant address space with wave-uniform addresses (so
// they become scalar loads into SGPRs); every step of a cell is the same
// arithmetic in the two-launch and in the blocked kernels (explicit fma, no
// contraction), so both produce bit-identical results.  Indices are 32-bit
// (the host rejects grids where M * nx or the step count reach 2^31).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "engine.hpp"
#include "launch.hpp"

namespace mb {
namespace {

constexpr int kTileSources = 4;  // sources per tile staged in LDS
constexpr int kMaxChunk = 256;   // steps per blocked launch
// fixed-point iterations of a strong-coupling E update, started from the
// cell's previous polarization current: each iteration gains about 4.5
// decimal digits on the Lambda workload (oracle: 4e-3, 2e-7, 9e-12, 5e-16
// relative changes from a zero start), so two reach FP32 and three FP64.
// With the exact field step the update takes Newton steps instead (the
// derivative of the phases in the field is known in closed form), whose
// error falls quadratically from the warm start: one for FP32, two for FP64.
template <typename R>
constexpr int strong_iters() { return sizeof(R) == 4 ? 2 : 3; }
template <typename R>
constexpr int strong_newton() { return sizeof(R) == 4 ? 1 : 2; }

// 1 / d for a Newton step (FP32: the hardware reciprocal, whose rounding only
// perturbs the step's size, not the equation it solves)
__device__ __forceinline__ float newton_gain(float d) { return __builtin_amdgcn_rcpf(d); }
__device__ __forceinline__ double newton_gain(double d) { return 1.0 / d; }

// Neighbour values within one wave by DPP wavefront shifts (lane l receives
// lane l+1, respectively l-1; the lane at the end of the wave receives 0).
__device__ __forceinline__ int dpp_from_right(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, false); }
__device__ __forceinline__ int dpp_from_left(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, false); }
__device__ __forceinline__ float lane_from_right(float v) { return __int_as_float(dpp_from_right(__float_as_int(v))); }
__device__ __forceinline__ float lane_from_left(float v) { return __int_as_float(dpp_from_left(__float_as_int(v))); }
__device__ __forceinline__ double lane_from_right(double v) {
  return __hiloint2double(dpp_from_right(__double2hiint(v)), dpp_from_right(__double2loint(v)));
}
__device__ __forceinline__ double lane_from_left(double v) {
  return __hiloint2double(dpp_from_left(__double2hiint(v)), dpp_from_left(__double2loint(v)));
}

// Register copy of the quantum coefficients of one material, indexed like
// the table (offset kCoefKap).
template <typename R, int SQ>
struct RegCoef {
  const R (&a)[SQ];
  __device__ __forceinline__ R operator[](int i) const { return a[i - kCoefKap]; }
};

template <typename T>
using cptr = const __attribute__((address_space(4))) T *;

template <typename T>
__device__ __forceinline__ cptr<T> kconst(const void *p) {
  return (cptr<T>)(p);
}

// (cos t - 1, sin t) of a field phase.  Small angles (the usual case: the
// phase per step is E dt (lam_j - lam_k)/hbar, a few 1e-2 rad) use the
// Taylor series truncated where the remainder drops below half an ulp;
// larger ones use angle halving and doubling (FP64) or the library sincos of
// t/2 with cos t - 1 = -2 sin^2(t/2) (FP32).
__device__ __forceinline__ void phase_taylor(double t, double &cm, double &sn) {
  const double t2 = t * t;
  double s = fma(t2, -1.0 / 6227020800.0, 1.0 / 39916800.0);
  s = fma(t2, s, -1.0 / 362880.0);
  s = fma(t2, s, 1.0 / 5040.0);
  s = fma(t2, s, -1.0 / 120.0);
  s = fma(t2, s, 1.0 / 6.0);
  sn = fma(-t * t2, s, t);  // t - t^3 (1/3! - t^2/5! + ...)
  double c = fma(t2, 1.0 / 87178291200.0, -1.0 / 479001600.0);
  c = fma(t2, c, 1.0 / 3628800.0);
  c = fma(t2, c, -1.0 / 40320.0);
  c = fma(t2, c, 1.0 / 720.0);
  c = fma(t2, c, -1.0 / 24.0);
  c = fma(t2, c, 0.5);
  cm = -t2 * c;             // -(t^2/2! - t^4/4! + ...)
}

// |t| <= 1/16: the series to t^5 and t^6 leave relative remainders of at
// most 1.2e-11 and 3e-12 (the terms t^7/7! and t^8/8!), far below FP32's ulp
constexpr float kPhaseShort = 0.0625f;
__device__ __forceinline__ void phase_short(float t, float &cm, float &sn) {
  const float t2 = t * t;
  const float s = fmaf(t2, 1.0f / 120.0f, -1.0f / 6.0f);
  sn = fmaf(t * t2, s, t);
  float c = fmaf(t2, -1.0f / 720.0f, 1.0f / 24.0f);
  c = fmaf(t2, c, -0.5f);
  cm = t2 * c;
}

__device__ __forceinline__ void phase_long(float t, float &cm, float &sn) {
  const float t2 = t * t;
  float s = fmaf(t2, 1.0f / 362880.0f, -1.0f / 5040.0f);
  s = fmaf(t2, s, 1.0f / 120.0f);
  s = fmaf(t2, s, -1.0f / 6.0f);
  sn = fmaf(t * t2, s, t);
  float c = fmaf(t2, -1.0f / 3628800.0f, 1.0f / 40320.0f);
  c = fmaf(t2, c, -1.0f / 720.0f);
  c = fmaf(t2, c, 1.0f / 24.0f);
  c = fmaf(t2, c, -0.5f);
  cm = t2 * c;
}

// |t| > 0.25 in FP64: the series at t / 2^k (below 0.25), then k double-angle
// steps, cos 2x - 1 = 2 c (c + 2) and sin 2x = 2 s (c + 1) for c = cos x - 1,
// s = sin x (no cancellation); each step doubles the absolute error, about
// 2^k ulp in all.  A short loop in few registers: the library sincos needed
// so many that the FP64 tiles spilled into accumulation registers.
// (k = 0 for the lanes with |t| <= 0.25)
__device__ __forceinline__ void phase_general(double t, double &cm, double &sn) {
  int k = 0;
  double ts = t;
  if (!(fabs(t) <= 0.25)) {
    const int e = ilogb(t);  // |t| < 2^(e+1)
    k = e > 61 ? 64 : (e < -2 ? 1 : e + 3);
    ts = ldexp(t, -k);
  }
  double c, s;
  phase_taylor(ts, c, s);
  for (int i = 0; i < k; ++i) {
    const double c2 = 2.0 * c * (c + 2.0);
    s = 2.0 * s * (c + 1.0);
    c = c2;
  }
  cm = c;
  sn = s;
}

// per lane: the short series, the long one, or sincos (the result depends on
// t alone, not on which lanes share the wave)
__device__ __forceinline__ void phase_taylor(float t, float &cm, float &sn) {
  if (fabsf(t) <= kPhaseShort)
    phase_short(t, cm, sn);
  else
    phase_long(t, cm, sn);
}

__device__ __forceinline__ void phase_general(float t, float &cm, float &sn) {
  if (fabsf(t) <= 0.5f) {
    phase_taylor(t, cm, sn);
  } else {
    float s, c;
    sincosf(0.5f * t, &s, &c);
    sn = 2.0f * s * c;
    cm = -2.0f * s * s;
  }
}

// the whole wave takes the polynomial without a divergent branch when every
// active lane's angle is small (the usual case); per-lane choice otherwise
template <typename R>
__device__ __forceinline__ void phase(R t, R &cm, R &sn) {
  if constexpr (sizeof(R) == 4) {
    if (__builtin_amdgcn_ballot_w64(!(fabsf(t) <= kPhaseShort)) == 0) {
      phase_short(t, cm, sn);
      return;
    }
  }
  const R lim = sizeof(R) == 8 ? R(0.25) : R(0.5);
  if (__builtin_amdgcn_ballot_w64(!(fabs(t) <= lim)) == 0)
    phase_taylor(t, cm, sn);
  else
    phase_general(t, cm, sn);
}

// Work of a cell's density update shared out over L wave groups: the
// eigenbasis coherence pairs (their two rows of z), the stored populations and
// the pairs of state rows (Re, Im of one coherence, kept together), each given
// in turn to the least loaded group (costs in multiply-adds of the general or
// the block form).
template <int N, int L, bool BK = false>
struct Split {
  static constexpr int M = mat_m(N);
  static constexpr int K = mat_k(N);
  static constexpr int P = N > 0 ? N * (N - 1) / 2 : 0;
  static constexpr int NP = N > 0 ? N - 1 : 0;
  static constexpr int kItems = 2 * P + NP;
  // item u < P: z pair u; P + a: population row a; P + NP + r: rows of pair r
  struct Table {
    int who[kItems > 0 ? kItems : 1];
  };
  static constexpr Table make_table() {
    Table t{};
    int load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int u = 0; u < kItems; ++u) {
      const int cost = u < P ? (BK ? NP + 2 * P : 2 * M) : u < P + NP ? (BK ? NP : M + K) : (BK ? 2 * P + 4 : 2 * (M + K));
      int best = 0;
      for (int g = 1; g < L; ++g)
        if (load[g] < load[best]) best = g;
      load[best] += cost;
      t.who[u] = best;
    }
    return t;
  }
  static constexpr Table kTable = make_table();
  static constexpr int owner(int item) { return L == 1 ? 0 : kTable.who[item]; }
  static constexpr int row_item(int a) { return a < NP ? P + a : P + NP + (a - NP) / 2; }
  // sub: the wave group (a constant, or a wave-uniform value for kernels
  // whose wave groups share one copy of the code)
  static constexpr bool owns(int sub, int a) { return L == 1 || owner(row_item(a)) == sub; }
  static constexpr bool owns_z(int sub, int r) { return L == 1 || owner(r / 2) == sub; }
  static constexpr bool owns_pop(int sub) {
    for (int a = 0; a < NP; ++a)
      if (owns(sub, a)) return true;
    return false;
  }
};

template <int N, typename R, bool BK = false>
struct Cell {
  static constexpr int M = mat_m(N);
  static constexpr int MA = M > 0 ? M : 1;
  static constexpr int K = mat_k(N);
  static constexpr int KA = K > 0 ? K : 1;
  static constexpr int P = K / 2;
  static constexpr int NP = N > 0 ? N - 1 : 0;
  // FP32 keeps, beside each state entry, the part of its running sum that the
  // FP32 rounding dropped (compensated summation): an entry that relaxes by
  // increments far below its own ulp, as slow populations do over 1e4..1e6
  // steps, would otherwise stall or drift by half an ulp per step
  static constexpr bool KC = sizeof(R) == 4 && N > 0;
  static constexpr int CA = KC ? MA : 1;

  // x_a <- x_a + inc (FP32: with the compensation xc_a)
  static __device__ __forceinline__ void add_inc(R &xa, R (&xc)[CA], int a, R inc) {
    if constexpr (KC) {
      const R y = inc - xc[a];
      const R t = xa + y;
      xc[a] = (t - xa) - y;
      xa = t;
    } else {
      xa = xa + inc;
    }
  }

  // entry t of the vector (x, d): the state, then the field increments
  static __device__ __forceinline__ R xd(const R (&x)[MA], const R (&d)[KA], int t) { return t < M ? x[t] : d[t - M]; }

  // z <- t0 + tm x: (Re, Im) of the coherences of the state in the dipole
  // eigenbasis (with L > 1 the rows of the pairs owned by group SUB); in the
  // block form Re z from the populations and the real parts of x, Im z from
  // the imaginary parts
  template <int L = 1, typename C>
  static __device__ __forceinline__ void coherences(const R (&x)[MA], R (&z)[KA], const C &mt, int sub = 0) {
    if constexpr (BK) {
#pragma unroll
      for (int q = 0; q < P; ++q) {
        if (!Split<N, L, BK>::owns_z(sub, 2 * q)) continue;
        R zr = mt[bk_t0(N) + q], zi = R(0);
#pragma unroll
        for (int a = 0; a < NP; ++a) zr = fma(mt[bk_tp(N) + q * NP + a], x[a], zr);
#pragma unroll
        for (int r = 0; r < P; ++r) {
          zr = fma(mt[bk_tr(N) + q * P + r], x[NP + 2 * r], zr);
          zi = fma(mt[bk_ti(N) + q * P + r], x[NP + 2 * r + 1], zi);
        }
        z[2 * q] = zr;
        z[2 * q + 1] = zi;
      }
    } else {
#pragma unroll
      for (int r = 0; r < K; ++r) {
        if (!Split<N, L, BK>::owns_z(sub, r)) continue;
        R acc = mt[coef_t0(N) + r];
#pragma unroll
        for (int j = 0; j < M; ++j) acc = fma(mt[coef_tm(N) + r * M + j], x[j], acc);
        z[r] = acc;
      }
    }
  }

  // z <- d = (e^{i theta_jk} - 1) z_jk: the change of eigenbasis coherence
  // (j, k), j < k, under the field conjugation, theta_jk = dt E (lam_j -
  // lam_k)/hbar, the sum of the consecutive angles E kappa_q; each phase is
  // carried as (cos - 1, sin), so the increment has no cancellation.
  // cay: the Cayley approximant of the field exponential instead: level j's
  // factor (1 + i x_j)/(1 - i x_j), x_j = E sigma_j / 2, so the consecutive
  // pair (q, q+1) turns by u/conj(u), u = 1 + x_q x_{q+1} + i (x_q - x_{q+1}):
  // cos - 1 = -2 d^2/|u|^2 and sin = 2 s d/|u|^2 with d = x_q - x_{q+1} and
  // s = 1 + x_q x_{q+1} (no cancellation for small angles).
  static constexpr int PA = P > 0 ? P : 1;

  // (cos - 1, sin) of every pair's angle, pair index k(k-1)/2 + j
  template <typename C>
  static __device__ __forceinline__ void pair_phases(R e, const C &mt, bool cay, R (&pcq)[PA], R (&psq)[PA]) {
    if constexpr (N >= 2) {
      R cm[N - 1], sn[N - 1];
      if (cay) {
#pragma unroll
        for (int q = 0; q < N - 1; ++q) {
          const R a = R(0.5) * e * mt[sigma_of(N, BK) + q], b = R(0.5) * e * mt[sigma_of(N, BK) + q + 1];
          const R dd = a - b, s = fma(a, b, R(1));
          const R inv = R(1) / fma(s, s, dd * dd);
          cm[q] = R(-2) * (dd * dd) * inv;
          sn[q] = R(2) * (s * dd) * inv;
        }
      } else {
#pragma unroll
        for (int q = 0; q < N - 1; ++q) phase(e * mt[kCoefKap + q], cm[q], sn[q]);
      }
#pragma unroll
      for (int j = 0; j < N - 1; ++j) {
        R pc = cm[j], ps = sn[j];
#pragma unroll
        for (int k = j + 1; k < N; ++k) {
          if (k > j + 1) {
            // (1 + pc + i ps)(1 + c2 + i s2) - 1
            const R c2 = cm[k - 1], s2 = sn[k - 1];
            const R nc = fma(pc, c2, fma(-ps, s2, pc + c2));
            const R ns = fma(ps, c2, fma(pc, s2, ps + s2));
            pc = nc;
            ps = ns;
          }
          pcq[k * (k - 1) / 2 + j] = pc;
          psq[k * (k - 1) / 2 + j] = ps;
        }
      }
    }
  }

  // z <- d = (e^{i theta_jk} - 1) z_jk with the pairs' (cos - 1, sin)
  static __device__ __forceinline__ void rotate_by(R (&z)[KA], const R (&pcq)[PA], const R (&psq)[PA]) {
#pragma unroll
    for (int q = 0; q < P; ++q) {
      const R re = z[2 * q], im = z[2 * q + 1];
      z[2 * q] = fma(re, pcq[q], -(im * psq[q]));
      z[2 * q + 1] = fma(re, psq[q], im * pcq[q]);
    }
  }

  // z <- d = (e^{i theta_jk} - 1) z_jk: the change of eigenbasis coherence
  // (j, k), j < k, under the field conjugation, theta_jk = dt E (lam_j -
  // lam_k)/hbar, the sum of the consecutive angles E kappa_q; each phase is
  // carried as (cos - 1, sin), so the increment has no cancellation.
  // cay: the Cayley approximant of the field exponential instead: level j's
  // factor (1 + i x_j)/(1 - i x_j), x_j = E sigma_j / 2, so the consecutive
  // pair (q, q+1) turns by u/conj(u), u = 1 + x_q x_{q+1} + i (x_q - x_{q+1}):
  // cos - 1 = -2 d^2/|u|^2 and sin = 2 s d/|u|^2 with d = x_q - x_{q+1} and
  // s = 1 + x_q x_{q+1} (no cancellation for small angles).
  template <typename C>
  static __device__ __forceinline__ void increments(R (&z)[KA], R e, const C &mt, bool cay = false) {
    if constexpr (N >= 2) {
      R pcq[PA], psq[PA];
      pair_phases(e, mt, cay, pcq, psq);
      rotate_by(z, pcq, psq);
    }
  }

  // polarization current n3D tr{mu L0(rho^{n+1/2})} = p0 + at . x + as . d
  // (two interleaved partial sums for instruction-level parallelism)
  template <typename C>
  static __device__ __forceinline__ R polar(const R (&x)[MA], const R (&d)[KA], const C &mt) {
    R acc0 = mt[coef_p0(N)], acc1 = R(0);
#pragma unroll
    for (int t = 0; t + 1 < M + K; t += 2) {
      acc0 = fma(mt[coef_at(N) + t], xd(x, d, t), acc0);
      acc1 = fma(mt[coef_at(N) + t + 1], xd(x, d, t + 1), acc1);
    }
    if constexpr ((M + K) % 2 == 1) acc0 = fma(mt[coef_at(N) + M + K - 1], xd(x, d, M + K - 1), acc0);
    return acc0 + acc1;
  }

  // sigma_{n+1} = e^{L0 dt} (x + S d): x_i <- x_i + (bf_i + (A - I)_i x +
  // (A S)_i d); with L > 1 the rows owned by group SUB (the others are left
  // as they are).  Block form: y = x + S d by its real and imaginary parts,
  // then x <- y + (bfp + ap y) on the populations and y + b y on each pair.
  template <int L = 1, typename C>
  static __device__ __forceinline__ void propagate(R (&x)[MA], R (&xc)[CA], const R (&d)[KA], const C &mt,
                                                   int sub = 0) {
    using SP = Split<N, L, BK>;
    if constexpr (BK) {
      // each row gains x + (increment): the small terms are summed on their own
      if (SP::owns_pop(sub)) {
        R dp[NP > 0 ? NP : 1], yp[NP > 0 ? NP : 1];
#pragma unroll
        for (int a = 0; a < NP; ++a) {
          R acc = R(0);
#pragma unroll
          for (int q = 0; q < P; ++q) acc = fma(mt[bk_sp(N) + a * P + q], d[2 * q], acc);
          dp[a] = acc;
          yp[a] = x[a] + acc;
        }
#pragma unroll
        for (int a = 0; a < NP; ++a) {
          if (!SP::owns(sub, a)) continue;
          R acc = mt[bk_bf(N) + a];
#pragma unroll
          for (int b = 0; b < NP; ++b) acc = fma(mt[bk_ap(N) + a * NP + b], yp[b], acc);
          add_inc(x[a], xc, a, dp[a] + acc);
        }
      }
#pragma unroll
      for (int r = 0; r < P; ++r) {
        if (!SP::owns(sub, NP + 2 * r)) continue;
        R dr = R(0), di = R(0);
#pragma unroll
        for (int q = 0; q < P; ++q) {
          dr = fma(mt[bk_sr(N) + r * P + q], d[2 * q], dr);
          di = fma(mt[bk_si(N) + r * P + q], d[2 * q + 1], di);
        }
        const R yr = x[NP + 2 * r] + dr, yi = x[NP + 2 * r + 1] + di;
        const R b0 = mt[bk_blk(N) + 4 * r], b1 = mt[bk_blk(N) + 4 * r + 1];
        const R b2 = mt[bk_blk(N) + 4 * r + 2], b3 = mt[bk_blk(N) + 4 * r + 3];
        add_inc(x[NP + 2 * r], xc, NP + 2 * r, dr + fma(b0, yr, b1 * yi));
        add_inc(x[NP + 2 * r + 1], xc, NP + 2 * r + 1, di + fma(b2, yr, b3 * yi));
      }
    } else {
      R inc[MA];
#pragma unroll
      for (int i = 0; i < M; ++i) {
        if (!SP::owns(sub, i)) continue;
        R acc = mt[coef_bf(N) + i];
#pragma unroll
        for (int t = 0; t < M + K; ++t) acc = fma(mt[coef_am(N) + i * (M + K) + t], xd(x, d, t), acc);
        inc[i] = acc;
      }
#pragma unroll
      for (int i = 0; i < M; ++i)
        if (SP::owns(sub, i)) add_inc(x[i], xc, i, inc[i]);
    }
  }

  // FP64 readout r0 + r . x + rs . d of a density quantity of rho^{n+1/2}
  static __device__ __forceinline__ double readout(const R (&x)[MA], const R (&d)[KA],
                                                   const double *__restrict__ ro) {
    double acc = ro[0];
#pragma unroll
    for (int t = 0; t < M + K; ++t) acc = fma(ro[1 + t], double(xd(x, d, t)), acc);
    return acc;
  }
};

__device__ __forceinline__ bool due(uint32_t n1, int64_t interval) { return n1 % uint32_t(interval) == 0u; }

template <int N, typename R>
__device__ __forceinline__ void record_density_all(const DevSim &sim, int c, uint32_t n1, int mat,
                                                const R (&x)[Cell<N, R>::MA], const R (&d)[Cell<N, R>::KA]) {
  for (int32_t r = 0; r < sim.n_rec_all; ++r) {
    const DevRecord &rc = sim.rec[sim.rec_all[r]];
    if (rc.quantity < 2 || !due(n1, rc.interval)) continue;
    rc.out[size_t(n1 / uint32_t(rc.interval) - 1) * size_t(sim.nx) + c] =
        Cell<N, R>::readout(x, d, rc.readout + mat * ro_len(N));
  }
}

// density records of one cell after local step n1 - 1 (values of rho^{n+1/2}):
// entries [rb, re) of the per-cell record table, then the whole-domain records
template <int N, typename R>
__device__ __forceinline__ void record_density(const DevSim &sim, int c, uint32_t n1, int mat,
                                            const R (&x)[Cell<N, R>::MA], const R (&d)[Cell<N, R>::KA], int rb,
                                            int re) {
  for (int32_t r = rb; r < re; ++r) {
    const DevRecord &rc = sim.rec_cell[r];
    if (rc.quantity < 2 || !due(n1, rc.interval)) continue;
    rc.out[n1 / uint32_t(rc.interval) - 1] = Cell<N, R>::readout(x, d, rc.readout + mat * ro_len(N));
  }
  record_density_all<N, R>(sim, c, n1, mat, x, d);
}

// value of a field record (E^{n+1}, H^{n+1/2}; density quantities read zero
// outside quantum cells); false for density quantities of quantum cells.  h is
// H in A/m (the kernels carry eta0 H, see DevSim::h_scale)
template <typename R>
__device__ __forceinline__ bool field_value(int quantity, R e, double h, bool qm, double &v) {
  if (quantity == 0) {
    v = double(e);
    return true;
  }
  if (quantity == 1) {
    v = h;
    return true;
  }
  if (!qm) {
    v = 0.0;
    return true;
  }
  return false;
}

template <typename R>
__device__ __forceinline__ void record_fields_all(const DevSim &sim, int c, uint32_t n1, R e, double h, bool qm) {
  for (int32_t r = 0; r < sim.n_rec_all; ++r) {
    const DevRecord &rc = sim.rec[sim.rec_all[r]];
    double v;
    if (!due(n1, rc.interval) || !field_value(rc.quantity, e, h, qm, v)) continue;
    rc.out[size_t(n1 / uint32_t(rc.interval) - 1) * size_t(sim.nx) + c] = v;
  }
}

template <typename R>
__device__ __forceinline__ void record_fields(const DevSim &sim, int c, uint32_t n1, R e, double h, bool qm, int rb,
                                              int re) {
  for (int32_t r = rb; r < re; ++r) {
    const DevRecord &rc = sim.rec_cell[r];
    double v;
    if (!due(n1, rc.interval) || !field_value(rc.quantity, e, h, qm, v)) continue;
    rc.out[n1 / uint32_t(rc.interval) - 1] = v;
  }
  record_fields_all(sim, c, n1, e, h, qm);
}

// Single-cell records of one tile's owned cells, copied to LDS at the start
// of a launch together with the readout row of each record's cell, so that a
// recording step reads no record descriptors from global memory.  A record's
// interval is a multiple `mult` of the simulation's record period (the gcd of
// all intervals); at the q-th multiple of the period (n1 = q * period) a
// record is due when q % mult == 0 and takes sample q / mult - 1.
constexpr int kTileRecs = 16;

template <int N>
struct TileRecs {
  static constexpr int RO = ro_len(N);
  double *out[kTileRecs];
  int64_t n_out[kTileRecs];  // samples the output holds
  uint32_t mult[kTileRecs];
  int32_t quantity[kTileRecs];
  double ro[kTileRecs][RO];

  // entry i <- record table entry r (one thread per entry)
  __device__ __forceinline__ void stage(const DevSim &sim, int i, int r) {
    const DevRecord &rc = sim.rec_cell[r];
    out[i] = rc.out;
    n_out[i] = sim.n_steps / rc.interval;
    mult[i] = uint32_t(rc.interval / sim.rec_every);
    quantity[i] = rc.quantity;
    if (rc.quantity >= 2 && rc.readout) {
      const double *row = rc.readout + int(sim.mat_e[rc.cell]) * RO;
      for (int a = 0; a < RO; ++a) ro[i][a] = row[a];
    }
  }

  // sample index of entry r at the q-th record period, or -1 when not due
  // (or, defensively, outside the output)
  __device__ __forceinline__ int64_t sample(int r, uint32_t q) const {
    const uint32_t m = mult[r];
    const int64_t at = m == 1u ? int64_t(q) - 1 : q % m == 0u ? int64_t(q / m) - 1 : -1;
    return at < n_out[r] ? at : -1;
  }

  // same arithmetic as Cell::readout; entries rb, rb + step, ... below re
  template <typename R, int MA, int KA>
  __device__ __forceinline__ void density(uint32_t q, const R (&x)[MA], const R (&d)[KA], int rb, int re,
                                          int step) const {
    constexpr int M = mat_m(N);
    for (int r = rb; r < re; r += step) {
      if (quantity[r] < 2) continue;
      const int64_t at = sample(r, q);
      if (at < 0) continue;
      double acc = ro[r][0];
#pragma unroll
      for (int t = 0; t < RO - 1; ++t) acc = fma(ro[r][1 + t], double(t < M ? x[t] : d[t - M]), acc);
      out[r][at] = acc;
    }
  }

  template <typename R>
  __device__ __forceinline__ void fields(uint32_t q, R e, double h, bool qm, int rb, int re, int step) const {
    for (int r = rb; r < re; r += step) {
      const int qty = quantity[r];
      if (qty >= 2 && qm) continue;  // density record of a quantum cell: written by density()
      const int64_t at = sample(r, q);
      double v;
      if (at < 0 || !field_value(qty, e, h, qm, v)) continue;
      out[r][at] = v;
    }
  }
};

// the cell's entries [rb, re) in the per-cell record table
__device__ __forceinline__ void record_range(const DevSim &sim, int c, int &rb, int &re) {
  rb = re = 0;
  if (sim.rec_first) {
    rb = sim.rec_first[c];
    re = sim.rec_first[c + 1];
  }
}

template <typename R>
__device__ __forceinline__ R apply_sources(const DevSim &sim, int c, uint32_t n1, R e) {
  for (int32_t j = 0; j < sim.n_src; ++j) {
    const DevSource &s = sim.src[j];
    if (int(s.cell) != c) continue;
    const R v = R(s.table[n1]);
    e = s.hard ? v : e + v;
  }
  return e;
}

// ---------------------------------------------------------------------------
// Temporally blocked kernel: one workgroup owns T = B - 2*halo consecutive
// cells of one simulation, loads them with `halo` extra cells on both sides,
// advances up to k <= halo steps with neighbour values exchanged through LDS
// (the valid region shrinks by one cell per side and step, as the redundant
// computation of overlapped tiles), and writes the owned cells to the other
// state buffer.  With L > 1 the workgroup holds L waves per 64 cells: every
// wave group keeps E and H of all B cells (the field updates are repeated)
// and computes only its own eigenbasis coherences and rows of the density
// state; both are exchanged through LDS every step (one barrier each), so
// each group sees the whole state and all field increments for the
// polarization, the records and its rows of the propagator.  The arithmetic
// per cell is the same for every B, L and coefficient placement.
// ---------------------------------------------------------------------------
template <int N, typename R, int B, int L>
struct TileShared {
  static constexpr int GM = L > 1 ? mat_m(N) : 1;
  static constexpr int GK = L > 1 && N > 0 ? mat_k(N) : 1;
  static constexpr int GB = L > 1 ? B : 1;
  R se[2][B], se2[B];  // E exchange (double-buffered by step parity), Mur exchange
  R src[kTileSources][kMaxChunk];
  TileRecs<N> trec;
  // density rows and eigenbasis coherences of every cell (L > 1).  One buffer
  // each suffices: the rows are read after a step's first barrier and
  // rewritten after its second, the coherences written after the first and
  // read after the second.
  R sx[GM][GB];
  R sz[GK][GB];
  int stop;         // a neighbour wait gave up: the tile ends the launch
};

// Device-coherent (agent-scope) accesses: they bypass the per-XCD caches, so
// tiles on different XCDs exchange cells without cache write-back or
// invalidation.  Used for the state a persistent launch hands between chunks.
template <typename T>
__device__ __forceinline__ T load_coherent(const T *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void store_coherent(T *p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// true once both neighbour tiles (and tile `self` when >= 0) have finished
// the chunk of epoch `target`; false after cs.spin_ticks of the device wall
// clock (the launch is then abandoned and the simulation's status reports it)
__device__ __forceinline__ bool neighbours_reached(const ChunkSync &cs, const DevTile &tile, uint32_t target,
                                                   int self = -1) {
  const int64_t t0 = wall_clock64();
  for (;;) {
    bool ok = true;
    if (self >= 0)
      ok = int32_t(__hip_atomic_load(cs.flags + self, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - target) >= 0;
    if (ok && tile.left >= 0)
      ok = int32_t(__hip_atomic_load(cs.flags + tile.left, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - target) >= 0;
    if (ok && tile.right >= 0)
      ok = int32_t(__hip_atomic_load(cs.flags + tile.right, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - target) >= 0;
    if (ok) return true;
    if (wall_clock64() - t0 > cs.spin_ticks) return false;
    __builtin_amdgcn_s_sleep(2);
  }
}

// wave groups (L > 1) that share one copy of the step code, the group being a
// wave-uniform run-time value: six or more levels in the general form, whose
// step (thousands of instructions) is too long for a copy per group to stay
// in the instruction cache (six-level QCL-like FP32 with a copy per group:
// 32 and 300 us per step with 2 and 4 groups against 11.9 us with one; with
// one shared copy 10.7 and 7.7 us).  Five levels keep a copy per group: the
// comb's 4-group tiles take 3.2 us per step so, 5.5 us with a shared copy.
template <int N, int L, bool BK>
constexpr bool shared_split() {
  return L > 1 && N >= 6 && !BK;
}

// tiles stay at <= 512 threads (a 1024-thread workgroup caps a wave at 128
// registers, below what most density updates need), except split FP32 tiles
// with up to 3 levels, whose waves fit in 128; five and six levels use at most
// 256 threads (their waves need the full register file)
template <int N, typename R, int B, int L>
constexpr bool shape_fits() {
  constexpr int max_threads = N >= 5 ? 256 : (N <= 3 && sizeof(R) == 4 && L > 1) ? 1024 : 512;
  return B * L <= max_threads && (L == 1 || (N >= 2 && (L < 8 || N >= 4))) &&
         sizeof(TileShared<N, R, B, L>) <= 65536;
}

// coefficients in registers: two levels, and three levels in FP32 with one
// wave per 64 cells and at most 256 cells (beyond that the registers spill)
template <int N, typename R, int B, int L>
constexpr bool regs_fit() {
  return N == 2 || (N == 3 && sizeof(R) == 4 && L == 1 && B <= 256);
}

// P: a persistent launch (several chunks, neighbour flags, device-coherent
// exchange of the owned cells); without it one chunk, and none of that code.
// tix: the tile.  Q: one item of a work-queue launch (P false), chunk qchunk
// of the launch: the tile first waits until it and both neighbours have
// finished chunk qchunk - 1, reads its cells with device-coherent loads and
// raises its flag when its stores are done.
template <int N, typename R, int B, int L, bool VC, int SUB, bool ST, bool P, bool CY, bool BK, bool Q = false>
__device__ __forceinline__ void tile_steps(const DevSim *__restrict__ sims, const DevTile *__restrict__ tiles,
                                           int tix, int qchunk, int64_t n0, int parity, int halo, int k,
                                           const ChunkSync &cs, TileShared<N, R, B, L> &sm, int rt_sub = 0) {
  using CL = Cell<N, R, BK>;
  using SP = Split<N, L, BK>;
  constexpr int M = CL::M, MA = CL::MA, S = stride_of(N, BK);
  constexpr bool WAVE = B == 64 && L == 1;  // one wave per tile: neighbours by DPP, no barriers
  // the wave group: SUB, or (kernels whose wave groups share one copy of the
  // step code, RT) the wave-uniform rt_sub
  constexpr bool RT = shared_split<N, L, BK>();
  const int sub = RT ? rt_sub : SUB;
  constexpr int SQ = S - kCoefKap;          // quantum part of a material's coefficients
  const DevTile tile = tiles[tix];
  // fields used inside the step loop are copied to locals below, so stores to
  // records cannot force them to be reloaded
  const DevSim &sim = sims[tile.sim];
  {
    // nothing to do in any chunk of this launch (the range is uniform over the tile)
    const int64_t first = n0 - sim.start, last = first + int64_t(P ? cs.n_chunks : 1) * k;
    if (last <= 0 || first >= sim.n_steps) return;
  }
  const int nx = int(sim.nx);
  const cptr<R> mtab = kconst<R>(sim.mtab);
  const int l = int(threadIdx.x) - sub * B;  // cell lane
  const int lo = tile.c0 - halo;
  const int c = lo + l;
  const bool in = c >= 0 && c < nx;
  const bool own = in && l >= halo && l < B - halo;
  int me = 0;
  R ca = 1, cbg = 0, cbd = 0, ch = 0;
  bool qm = false;
  if (in) {
    me = sim.mat_e[c];
    const int mh = sim.mat_h[c];
    ca = mtab[me * S + kCoefA];
    cbg = mtab[me * S + kCoefBG];
    cbd = mtab[me * S + kCoefBD];
    ch = mtab[mh * S + kCoefH];
    if constexpr (N > 0) qm = mtab[me * S + kCoefQM] != R(0);
  }
  // sources inside this tile: their values for each chunk are staged in LDS
  // (ordered before the first read by the first barrier of the step loop); a
  // lane knows the one staged source at its cell.  Tiles with more than
  // kTileSources sources, or two at one cell, read the source tables directly.
  int my_src = -1;
  bool my_hard = false;
  int staged_cell[kTileSources];
  const double *staged_tab[kTileSources];
  int n_ts = 0;
  bool src_direct = false;
  for (int j = 0; j < sim.n_src; ++j) {
    const DevSource sj = sim.src[j];
    const int cell = int(sj.cell);
    if (cell < lo || cell >= lo + B) continue;
    bool dup = false;
#pragma unroll
    for (int t = 0; t < kTileSources; ++t) dup = dup || (t < n_ts && staged_cell[t] == cell);
    if (n_ts == kTileSources || dup) {
      src_direct = true;
      break;
    }
#pragma unroll
    for (int t = 0; t < kTileSources; ++t)
      if (t == n_ts) {
        staged_cell[t] = cell;
        staged_tab[t] = sj.table;
      }
    if (cell == c) {
      my_src = n_ts;
      my_hard = sj.hard != 0;
    }
    ++n_ts;
  }
  const bool hcell = in && c <= nx - 2;
  const bool ecell = in && c >= 1 && c <= nx - 2;
  // H at the left node (cell c-1) is advanced here too, with the arithmetic
  // of the lane that owns it, so no exchange of H is needed
  const bool hleft = in && c >= 1;
  const R chl = hleft ? mtab[int(sim.mat_h[c - 1]) * S + kCoefH] : R(0);
  const bool left = in && nx > 1 && c == 0, right = in && nx > 1 && c == nx - 1;
  const bool mur_tile = nx > 1 && ((sim.edge_l == 1 && lo <= 0 && 0 < lo + B) ||
                                   (sim.edge_r == 1 && lo <= nx - 1 && nx - 1 < lo + B));
  const bool mur_l = left && sim.edge_l == 1, mur_r = right && sim.edge_r == 1;
  // the inner neighbour of a Mur edge cell is the next lane of the same wave
  // unless the edge cell is the last (left edge) or first (right edge) lane of
  // its wave: then the new E of the neighbour goes through LDS and a barrier
  const bool mur_dpp = (!(sim.edge_l == 1 && lo <= 0 && 0 < lo + B) || ((-lo) & 63) != 63) &&
                       (!(sim.edge_r == 1 && lo <= nx - 1 && nx - 1 < lo + B) || ((nx - 1 - lo) & 63) != 0);
  const bool pec = (left && sim.edge_l == 0) || (right && sim.edge_r == 0);
  const bool load_l = left && sim.edge_l == 2, load_r = right && sim.edge_r == 2;
  const R lg_l = R(sim.load_g_l), ld_l = R(sim.load_d_l), lg_r = R(sim.load_g_r), ld_r = R(sim.load_d_r);
  // the cell's entries in the per-cell record table, fetched once per launch;
  // when the tile's owned cells hold at most kTileRecs entries they are
  // staged in LDS (visible after the first barrier) and [rb, re) index there.
  // Staged records are shared out over the first RS wave groups (entry
  // rb + SUB, then every RS-th), the rest is written by the first wave group.
  // (Each group is its own copy of the step loop: with more than four groups,
  // or the long loops of 5 and 6 levels, copies with record code outgrow the
  // instruction cache, and there the records are a small part of a step.)
  constexpr int RS = N >= 5 ? 1 : L < 4 ? L : 4;
  int rb = 0, re = 0;
  bool rec_lds = false;
  bool rec_fld = false;  // this lane's entries hold one that the field records write
  if (sim.rec_first) {
    const int o0 = tile.c0, o1 = min(tile.c0 + B - 2 * halo, nx);
    const int rbase = sim.rec_first[o0], n_tr = sim.rec_first[o1] - rbase;
    rec_lds = n_tr <= kTileRecs;
    if (rec_lds && int(threadIdx.x) < n_tr) sm.trec.stage(sim, int(threadIdx.x), rbase + int(threadIdx.x));
    if (own && (rec_lds ? sub < RS : sub == 0)) {
      record_range(sim, c, rb, re);
      for (int r = rb + (rec_lds ? sub : 0); r < re; r += rec_lds ? RS : 1) {
        const int qty = sim.rec_cell[r].quantity;
        rec_fld = rec_fld || qty < 2 || !qm;  // E or H, or a density quantity outside the medium
      }
      if (rec_lds) {
        rb -= rbase;
        re -= rbase;
      }
    }
  }
  const bool rec_here = sub < RS && own && (re > rb || (sub == 0 && sim.n_rec_all > 0));
  const bool rec_fields_here = rec_here && (rec_fld || (sub == 0 && sim.n_rec_all > 0));
  const bool rec_tile = sim.rec_first != nullptr || sim.n_rec_all > 0;  // uniform
  const uint32_t rec_every = uint32_t(sim.rec_every);
  const double h_scale = sim.h_scale;
  const R kap_l = R(sim.kap_l), kap_r = R(sim.kap_r);
  // field part by the Cayley approximant (kernels of their own: the extra
  // phase code would cost the other kernels instruction-cache space)
  constexpr bool cay = CY;

  // coefficients of a single-material wave held in registers for the launch
  // (those this wave group reads: phases, polarization, its propagator rows)
  auto coef_used = [](int i) {
    const int t = i + kCoefKap;
    if (t >= sigma_of(N, BK)) return CY;  // Cayley coefficients (every wave group rotates)
    if (t < coef_bf(N) || BK) return true;  // phases and polarization; all of the (small) block form
    if (t < coef_am(N)) return SP::owns(SUB, t - coef_bf(N));
    if (t < coef_t0(N)) return SP::owns(SUB, (t - coef_am(N)) / prop_w(N));
    if (t < coef_tm(N)) return SP::owns_z(SUB, t - coef_t0(N));
    return SP::owns_z(SUB, (t - coef_tm(N)) / (M > 0 ? M : 1));
  };
  // (each lane holds its own cell's material, so waves across a material
  // boundary cost the same as single-material ones)
  R cf[VC ? SQ : 1];
  if constexpr (VC && N > 0) {
#pragma unroll
    for (int i = 0; i < SQ; ++i)
      if (coef_used(i)) cf[i] = qm ? mtab[me * S + kCoefKap + i] : R(0);
    // opaque register copies: keeps the compiler from re-loading the
    // coefficients from memory inside the step loop
#pragma unroll
    for (int i = 0; i < SQ; ++i)
      if (coef_used(i)) asm volatile("" : "+v"(cf[i]));
  }

  // runs f(coefficients, material) for the wave's quantum cells: once with
  // the lanes' register coefficients, or once per material present (scalar
  // loads of that material's coefficients) for the lanes of that material
  auto per_material = [&](auto &&f) {
    if constexpr (VC) {
      if (qm) f(RegCoef<R, VC ? SQ : 1>{cf}, me);
    } else {
      uint64_t todo = __ballot(qm);
      while (todo) {
        const int lead = __ffsll(static_cast<unsigned long long>(todo)) - 1;
        const int mm = __builtin_amdgcn_readlane(me, lead);
        const bool mine = qm && me == mm;
        if (mine) f(mtab + __builtin_amdgcn_readfirstlane(mm * S), mm);  // uniform: scalar loads
        todo &= ~__ballot(mine);
      }
    }
  };

  R e = 0, h = 0, hl = 0;
  R x[MA];
  R xc[CL::CA];     // FP32: the compensation of the owned state entries
  R z[CL::KA];      // eigenbasis coherences of x, then the field increments d
  double qn = 0.0;  // strong coupling: (n3D/dt) tr{mu rho^n} of the cell, carried in FP64
  R pprev = 0;      // strong coupling: the cell's last polarization current
  // strong coupling: tr{mu rho^{n+1}} as a function of the field angle,
  // sA + sum_q (sal_q (cos - 1) + sbe_q sin) over the pairs q
  double sA = 0.0, sal[ST ? CL::PA : 1], sbe[ST ? CL::PA : 1];

  // density rows of this wave group published for the other groups (L > 1);
  // they are read after the next step's E exchange barrier
  auto publish_x = [&]() {
    if constexpr (L > 1 && N > 0) {
#pragma unroll
      for (int a = 0; a < M; ++a)
        if (SP::owns(sub, a)) sm.sx[a][l] = x[a];
    }
  };

  const int n_chunks = P ? cs.n_chunks : 1;
  for (int chunk = 0; chunk < n_chunks; ++chunk) {
    const int64_t ls64 = n0 + int64_t(chunk) * k - sim.start;
    if (ls64 >= sim.n_steps) break;  // the simulation has finished (uniform over its tiles)
    if (ls64 < 0) continue;          // not started yet (uniform over its tiles)
    const int ls0 = int(ls64);
    const int ks = int(min(int64_t(k), sim.n_steps - ls64));
    const int par = parity ^ (chunk & 1) ^ sim.parity_off;
    const R *__restrict__ e_in = static_cast<const R *>(sim.e[par]);
    const R *__restrict__ h_in = static_cast<const R *>(sim.h[par]);
    const R *__restrict__ x_in = static_cast<const R *>(sim.x[par]);
    if (Q && qchunk > 0 && ls64 >= k) {
      // work-queue item whose simulation ran the previous chunk in this
      // launch: the tile's own and both neighbours' stores of that chunk
      // (other workgroups, handed out earlier) are complete first
      if (threadIdx.x == 0) {
        const bool ok = neighbours_reached(cs, tile, cs.epoch + uint32_t(qchunk), tix);
        sm.stop = !ok;
        if (!ok) atomicOr(sim.status, kStatusWaitTimeout);
      }
      __syncthreads();
      if (sm.stop) return;
    }
    // after the first chunk of a persistent launch the cells come from
    // neighbour tiles' stores of this launch: device-coherent loads
    const bool fresh = Q || (P && chunk > 0);
    auto ld = [fresh](const auto *ptr) { return fresh ? load_coherent(ptr) : *ptr; };
    e = h = hl = 0;
#pragma unroll
    for (int a = 0; a < MA; ++a) x[a] = 0;
#pragma unroll
    for (int a = 0; a < CL::CA; ++a) xc[a] = 0;
#pragma unroll
    for (int a = 0; a < CL::KA; ++a) z[a] = 0;
    if (in) {
      e = ld(e_in + c);
      h = ld(h_in + c);
      if constexpr (N > 0) {
        if (qm) {
#pragma unroll
          for (int a = 0; a < M; ++a)
            if (SP::owns(sub, a)) x[a] = ld(x_in + a * nx + c);
          if constexpr (CL::KC) {
#pragma unroll
            for (int a = 0; a < M; ++a)
              if (SP::owns(sub, a)) xc[a] = ld(x_in + (M + a) * nx + c);
          }
        }
      }
    }
    if constexpr (ST) {
      if (qm) {
        qn = ld(sim.qs[par] + c);
        pprev = R(ld(sim.qs[par] + 2 * nx + c));
      }
    }
    if (hleft) hl = ld(h_in + c - 1);
    for (int t = 0; t < n_ts; ++t)
      for (int q = int(threadIdx.x); q < ks; q += B * L) sm.src[t][q] = R(staged_tab[t][ls0 + q + 1]);
    // record periods: steps left before the next one, and its index
    uint32_t rec_in = rec_every - 1u - uint32_t(ls0) % rec_every;
    uint32_t rec_q = uint32_t(ls0) / rec_every + 1u;
    if constexpr (WAVE) __syncthreads();  // staged source values and records visible

    publish_x();

    for (int s = 0; s < ks; ++s) {
      const uint32_t n1 = uint32_t(ls0 + s + 1);
      const bool rec_step = rec_tile && rec_in == 0u;  // uniform: n1 is a multiple of the record period
      const uint32_t rq = rec_q;  // n1 / record period on a recording step
      rec_in = rec_in == 0u ? rec_every - 1u : rec_in - 1u;
      rec_q += rec_in == rec_every - 1u ? 1u : 0u;
      const int buf = s & 1;
      R er, el;
      if constexpr (WAVE) {
        er = lane_from_right(e);
        el = lane_from_left(e);
      } else {
        if (sub == 0) sm.se[buf][l] = e;
        __syncthreads();
        er = l + 1 < B ? sm.se[buf][l + 1] : R(0);
        el = l > 0 ? sm.se[buf][l - 1] : R(0);
      }
      if constexpr (L > 1 && N > 0) {
        if (qm) {
#pragma unroll
          for (int a = 0; a < M; ++a)
            if (!SP::owns(sub, a)) x[a] = sm.sx[a][l];
        }
      }
      h = hcell ? fma(ch, er - e, h) : h;
      hl = hleft ? fma(chl, e - el, hl) : hl;
      R p = 0;
      if constexpr (ST && N > 0) {
        // strong coupling: the E update of an interior quantum cell depends on
        // rho^{n+1}, driven by (E^n + E^{n+1})/2; fixed-point iteration from the
        // cell's previous polarization current.  The FP64 readout qt of (x, d),
        // d_q = (e^{i theta_q} - 1) z_q, is written out per pair once per step,
        // so an iteration costs the phases and 2 FP64 multiply-adds per pair.
        per_material([&](const auto &mt, int mm) {
          CL::coherences(x, z, mt);
          auto readout_terms = [&](const cptr<double> qt) {
            sA = qt[0];
#pragma unroll
            for (int t = 0; t < M; ++t) sA = fma(qt[1 + t], double(x[t]), sA);
#pragma unroll
            for (int q = 0; q < CL::P; ++q) {
              const double zr = double(z[2 * q]), zi = double(z[2 * q + 1]);
              const double qr = qt[1 + M + 2 * q], qi = qt[2 + M + 2 * q];
              sal[q] = fma(qr, zr, qi * zi);
              sbe[q] = fma(qi, zr, -(qr * zi));
            }
          };
          // the material's readout row: scalar loads when the wave's quantum
          // lanes share one material (always with scalar coefficient loads),
          // else the lane's own row (register coefficients: a wave may cross a
          // material boundary)
          const int m0 = __builtin_amdgcn_readfirstlane(mm);
          if (!VC || __builtin_amdgcn_ballot_w64(mm != m0) == 0)
            readout_terms(kconst<double>(sim.qtab) + m0 * ro_len(N));
          else
            readout_terms(kconst<double>(sim.qtab) + mm * ro_len(N));
          R pi = pprev;
          if constexpr (!CY) {
            // Newton on g(pi) = q(E_mid(pi)) - qn - pi, where E_mid = (E^n +
            // E^{n+1}(pi))/2 moves by -cbg/2 per unit pi and pair q's angle by
            // kq_q (its consecutive gaps' sum) per unit field:
            // dq/dE_mid = sum_q kq_q (sbe_q cos - sal_q sin)
            double kq[CL::PA];
#pragma unroll
            for (int j = 0; j + 1 < N; ++j) {
              double acc = 0.0;
#pragma unroll
              for (int k2 = j + 1; k2 < N; ++k2) {
                acc += double(mt[kCoefKap + k2 - 1]);
                kq[k2 * (k2 - 1) / 2 + j] = acc;
              }
            }
            for (int it = 0; it < strong_newton<R>(); ++it) {
              const R es = fma(cbd, h - hl, fma(ca, e, -(cbg * pi)));
              R pcq[CL::PA], psq[CL::PA];
              CL::pair_phases(R(0.5) * (e + es), mt, false, pcq, psq);
              double tq = sA, dq = 0.0;
#pragma unroll
              for (int q = 0; q < CL::P; ++q) {
                const double pc = double(pcq[q]), ps = double(psq[q]);
                tq = fma(sal[q], pc, fma(sbe[q], ps, tq));
                dq = fma(kq[q], fma(sbe[q], pc + 1.0, -(sal[q] * ps)), dq);
              }
              const R gain = newton_gain(fma(R(0.5) * cbg, R(dq), R(1)));  // -1 / g'(pi)
              pi = fma(R(tq - qn) - pi, gain, pi);
            }
          } else {
            for (int it = 0; it < strong_iters<R>(); ++it) {
              const R es = fma(cbd, h - hl, fma(ca, e, -(cbg * pi)));
              R pcq[CL::PA], psq[CL::PA];
              CL::pair_phases(R(0.5) * (e + es), mt, cay, pcq, psq);
              double tq = sA;
#pragma unroll
              for (int q = 0; q < CL::P; ++q) tq = fma(sal[q], double(pcq[q]), fma(sbe[q], double(psq[q]), tq));
              pi = R(tq - qn);
            }
          }
          p = pi;
        });
        pprev = p;
      } else if constexpr (N > 0) {
        auto finish = [&](const auto &mt, int mm) {
          CL::increments(z, e, mt, cay);
          p = CL::polar(x, z, mt);
          if (rec_step) {
            if (rec_here) {
              if (rec_lds) {
                sm.trec.density(rq, x, z, rb + sub, re, RS);
                if (sub == 0) record_density_all<N, R>(sim, c, n1, mm, x, z);
              } else {
                record_density<N, R>(sim, c, n1, mm, x, z, rb, re);
              }
            }
          }
          CL::template propagate<L>(x, xc, z, mt, sub);
        };
        if constexpr (L == 1) {
          per_material([&](const auto &mt, int mm) {
            CL::coherences(x, z, mt);
            finish(mt, mm);
          });
        } else {
          // this group's coherence rows, exchanged through LDS
          per_material([&](const auto &mt, int) { CL::template coherences<L>(x, z, mt, sub); });
#pragma unroll
          for (int r = 0; r < CL::K; ++r)
            if (SP::owns_z(sub, r)) sm.sz[r][l] = z[r];
          __syncthreads();
          if (qm) {
#pragma unroll
            for (int r = 0; r < CL::K; ++r)
              if (!SP::owns_z(sub, r)) z[r] = sm.sz[r][l];
          }
          per_material(finish);
        }
      }
      const R eo = e;
      e = ecell ? fma(cbd, h - hl, fma(ca, eo, -(cbg * p))) : e;
      if (mur_tile) {
        R enr, enl;
        if (WAVE || mur_dpp) {
          enr = lane_from_right(e);
          enl = lane_from_left(e);
        } else {
          if (sub == 0) sm.se2[l] = e;
          __syncthreads();
          enr = l + 1 < B ? sm.se2[l + 1] : R(0);
          enl = l > 0 ? sm.se2[l - 1] : R(0);
        }
        e = mur_l ? fma(kap_l, enr - eo, er) : e;
        e = mur_r ? fma(kap_r, enl - eo, el) : e;
      }
      e = pec ? R(0) : e;
      e = load_l ? fma(lg_l, eo, ld_l * h) : e;        // H_{1/2} is this lane's own
      e = load_r ? fma(lg_r, eo, -(ld_r * hl)) : e;    // H_{nx-3/2} is the tracked left node
      if (src_direct) {
        if (in) e = apply_sources(sim, c, n1, e);
      } else if (n_ts > 0) {
        if (my_src >= 0) {
          const R v = sm.src[my_src][s];
          e = my_hard ? v : e + v;
        }
      }
      if constexpr (ST && N > 0) {
        // rho^{n+1} with the final E^{n+1}: rotation by the midpoint field, the
        // new tr{mu rho}, records of rho^{n+1}, propagation of the running state
        per_material([&](const auto &mt, int mm) {
          R pcq[CL::PA], psq[CL::PA];
          CL::pair_phases(R(0.5) * (eo + e), mt, cay, pcq, psq);
          double tq = sA;
#pragma unroll
          for (int q = 0; q < CL::P; ++q) tq = fma(sal[q], double(pcq[q]), fma(sbe[q], double(psq[q]), tq));
          qn = tq;
          CL::rotate_by(z, pcq, psq);
          if (rec_step) {
            if (rec_here) {
              if (rec_lds) {
                sm.trec.density(rq, x, z, rb + sub, re, RS);
                if (sub == 0) record_density_all<N, R>(sim, c, n1, mm, x, z);
              } else {
                record_density<N, R>(sim, c, n1, mm, x, z, rb, re);
              }
            }
          }
          CL::propagate(x, xc, z, mt);
        });
      }
      if (rec_step) {
        if (rec_fields_here) {
          if (rec_lds) {
            sm.trec.fields(rq, e, hcell ? double(h) * h_scale : 0.0, qm, rb + sub, re, RS);
            if (sub == 0) record_fields_all(sim, c, n1, e, hcell ? double(h) * h_scale : 0.0, qm);
          } else {
            record_fields(sim, c, n1, e, hcell ? double(h) * h_scale : 0.0, qm, rb, re);
          }
        }
      }
      if (s + 1 < ks) publish_x();
    }
    if (own) {
      R *__restrict__ e_out = static_cast<R *>(sim.e[par ^ 1]);
      R *__restrict__ h_out = static_cast<R *>(sim.h[par ^ 1]);
      R *__restrict__ x_out = static_cast<R *>(sim.x[par ^ 1]);
      // persistent launches: device-coherent stores, read by the neighbours
      constexpr bool share = P || Q;
      auto st = [share](auto *ptr, auto v) {
        if (share)
          store_coherent(ptr, v);
        else
          *ptr = v;
      };
      if (sub == 0) {
        st(e_out + c, e);
        st(h_out + c, h);
      }
      if constexpr (N > 0) {
        if (qm) {
#pragma unroll
          for (int a = 0; a < M; ++a)
            if (SP::owns(sub, a)) st(x_out + a * nx + c, x[a]);
          if constexpr (CL::KC) {
#pragma unroll
            for (int a = 0; a < M; ++a)
              if (SP::owns(sub, a)) st(x_out + (M + a) * nx + c, xc[a]);
          }
          if constexpr (ST) {
            st(sim.qs[par ^ 1] + c, qn);
            st(sim.qs[par ^ 1] + 2 * nx + c, double(pprev));
          }
        }
      }
      if (sub == 0 && (!isfinite(double(e)) || !isfinite(double(h)))) atomicOr(sim.status, kStatusNonFinite);
    }
    if (Q) {
      // work-queue item done: every wave's coherent stores are complete
      // before the tile's flag is raised
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (threadIdx.x == 0) store_coherent(cs.flags + tix, cs.epoch + uint32_t(qchunk) + 1u);
    } else if (P && chunk + 1 < n_chunks) {
      // every wave's coherent stores of its owned cells are complete before
      // the tile's flag is raised; the next chunk's cells are read (coherent
      // loads) after both neighbours have raised theirs
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");  // keeps the stores above the wait
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (threadIdx.x == 0) {
        const uint32_t target = cs.epoch + uint32_t(chunk) + 1u;
        store_coherent(cs.flags + tix, target);
        const bool ok = neighbours_reached(cs, tile, target);
        sm.stop = !ok;
        if (!ok) atomicOr(sim.status, kStatusWaitTimeout);
      }
      __syncthreads();
      if (sm.stop) return;
    }
  }
}

// runs the specialisation of wave group `sub` (wave-uniform); every group
// executes the same sequence of barriers
template <int N, typename R, int B, int L, bool VC, bool P, bool CY, bool BK, int S = 0>
__device__ __forceinline__ void run_group(int sub, const DevSim *__restrict__ sims, const DevTile *__restrict__ tiles,
                                          int64_t n0, int parity, int halo, int k, const ChunkSync &cs,
                                          TileShared<N, R, B, L> &sm) {
  if constexpr (shared_split<N, L, BK>()) {
    tile_steps<N, R, B, L, VC, 0, false, P, CY, BK>(sims, tiles, blockIdx.x, -1, n0, parity, halo, k, cs, sm, sub);
  } else if constexpr (S + 1 < L) {
    if (sub == S)
      tile_steps<N, R, B, L, VC, S, false, P, CY, BK>(sims, tiles, blockIdx.x, -1, n0, parity, halo, k, cs, sm);
    else
      run_group<N, R, B, L, VC, P, CY, BK, S + 1>(sub, sims, tiles, n0, parity, halo, k, cs, sm);
  } else {
    tile_steps<N, R, B, L, VC, S, false, P, CY, BK>(sims, tiles, blockIdx.x, -1, n0, parity, halo, k, cs, sm);
  }
}

// ST: strong coupling (one wave per 64 cells only); CY: Cayley field step; BK:
// the block form of the density tables
template <int N, typename R, int B, int L, bool VC, bool ST, bool P, bool CY, bool BK>
__global__ void __launch_bounds__(B * L) k_blocked(const DevSim *__restrict__ sims,
                                                   const DevTile *__restrict__ tiles, int64_t n0, int parity,
                                                   int halo, int k, ChunkSync cs) {
  __shared__ TileShared<N, R, B, L> sm;
  if constexpr (L == 1) {
    tile_steps<N, R, B, 1, VC, 0, ST, P, CY, BK>(sims, tiles, blockIdx.x, -1, n0, parity, halo, k, cs, sm);
  } else {
    run_group<N, R, B, L, VC, P, CY, BK>(__builtin_amdgcn_readfirstlane(int(threadIdx.x) / B), sims, tiles, n0, parity,
                                         halo, k, cs, sm);
  }
}

// ---------------------------------------------------------------------------
// Two-launch step (Alg. 1 as written): the first kernel updates H, rho and p
// for every cell, the second E, the edges, the sources and the field records.
// E is double-buffered, H, rho and p are updated in place.
// ---------------------------------------------------------------------------
constexpr int kPlainBlock = 256;

template <int N, bool BK>
__global__ void __launch_bounds__(kPlainBlock) k_plain_hd(const DevSim *__restrict__ sims,
                                                          const DevTile *__restrict__ tiles, int64_t n0,
                                                          int parity) {
  using R = double;
  using CL = Cell<N, R, BK>;
  constexpr int M = CL::M, MA = CL::MA, S = stride_of(N, BK);
  const DevTile tile = tiles[blockIdx.x];
  const DevSim &sim = sims[tile.sim];
  const int64_t n64 = n0 - sim.start;
  if (n64 < 0 || n64 >= sim.n_steps) return;
  const uint32_t n1 = uint32_t(n64 + 1);
  const int nx = int(sim.nx);
  const int c = tile.c0 + int(threadIdx.x);
  if (c >= nx) return;
  const int par = parity ^ sim.parity_off;
  const R *__restrict__ e_in = static_cast<const R *>(sim.e[par]);
  R *__restrict__ hh = static_cast<R *>(sim.h[0]);
  R *__restrict__ xx = static_cast<R *>(sim.x[0]);
  R *__restrict__ pp = static_cast<R *>(sim.p);
  const cptr<R> mtab = kconst<R>(sim.mtab);
  const R e = e_in[c];
  if (c <= nx - 2) hh[c] = fma(mtab[sim.mat_h[c] * S + kCoefH], e_in[c + 1] - e, hh[c]);
  R p = 0;
  if constexpr (N > 0) {
    const int me = sim.mat_e[c];
    const bool qm = mtab[me * S + kCoefQM] != R(0);
    int rb = 0, re = 0;
    const bool rec_now = sim.n_rec > 0 && n1 % uint32_t(sim.rec_every) == 0u;
    if (rec_now) record_range(sim, c, rb, re);
    uint64_t todo = __ballot(qm);
    while (todo) {
      const int lead = __ffsll(static_cast<unsigned long long>(todo)) - 1;
      const int mm = __builtin_amdgcn_readlane(me, lead);
      const bool mine = qm && me == mm;
      if (mine) {
        const cptr<R> mt = mtab + __builtin_amdgcn_readfirstlane(mm * S);  // uniform: scalar loads
        R x[MA], z[CL::KA], xc[CL::CA];  // FP64: no compensation
#pragma unroll
        for (int a = 0; a < M; ++a) x[a] = xx[a * nx + c];
        CL::coherences(x, z, mt);
        CL::increments(z, e, mt, sim.cayley != 0);
        p = CL::polar(x, z, mt);
        if (rec_now) record_density<N, R>(sim, c, n1, mm, x, z, rb, re);
        CL::propagate(x, xc, z, mt);
#pragma unroll
        for (int a = 0; a < M; ++a) xx[a * nx + c] = x[a];
      }
      todo &= ~__ballot(mine);
    }
  }
  pp[c] = p;
}

__device__ __forceinline__ double plain_interior(const DevSim &sim, const double *__restrict__ e_in,
                                                 const double *__restrict__ hh, const double *__restrict__ pp,
                                                 cptr<double> mtab, int stride, int c) {
  const int me = sim.mat_e[c];
  const double ca = mtab[me * stride + kCoefA], cbg = mtab[me * stride + kCoefBG],
               cbd = mtab[me * stride + kCoefBD];
  return fma(cbd, hh[c] - hh[c - 1], fma(ca, e_in[c], -(cbg * pp[c])));
}

template <int N, bool BK>
__global__ void __launch_bounds__(kPlainBlock) k_plain_e(const DevSim *__restrict__ sims,
                                                         const DevTile *__restrict__ tiles, int64_t n0,
                                                         int parity) {
  using R = double;
  constexpr int S = stride_of(N, BK);
  const DevTile tile = tiles[blockIdx.x];
  const DevSim &sim = sims[tile.sim];
  const int64_t n64 = n0 - sim.start;
  if (n64 < 0 || n64 >= sim.n_steps) return;
  const uint32_t n1 = uint32_t(n64 + 1);
  const int nx = int(sim.nx);
  const int c = tile.c0 + int(threadIdx.x);
  if (c >= nx) return;
  const int par = parity ^ sim.parity_off;
  const R *__restrict__ e_in = static_cast<const R *>(sim.e[par]);
  R *__restrict__ e_out = static_cast<R *>(sim.e[par ^ 1]);
  const R *__restrict__ hh = static_cast<const R *>(sim.h[0]);
  const R *__restrict__ pp = static_cast<const R *>(sim.p);
  const cptr<R> mtab = kconst<R>(sim.mtab);
  R e = e_in[c];
  if (nx > 1) {
    if (c >= 1 && c <= nx - 2) {
      e = plain_interior(sim, e_in, hh, pp, mtab, S, c);
    } else if (c == 0) {
      e = sim.edge_l == 0   ? 0.0
          : sim.edge_l == 1 ? fma(sim.kap_l, plain_interior(sim, e_in, hh, pp, mtab, S, 1) - e_in[0], e_in[1])
                            : fma(sim.load_g_l, e_in[0], sim.load_d_l * hh[0]);
    } else {
      e = sim.edge_r == 0 ? 0.0
          : sim.edge_r == 1
              ? fma(sim.kap_r, plain_interior(sim, e_in, hh, pp, mtab, S, nx - 2) - e_in[nx - 1], e_in[nx - 2])
              : fma(sim.load_g_r, e_in[nx - 1], -(sim.load_d_r * hh[nx - 2]));
    }
  }
  e = apply_sources(sim, c, n1, e);
  e_out[c] = e;
  if (sim.n_rec > 0 && n1 % uint32_t(sim.rec_every) == 0u) {
    bool qm = false;
    if constexpr (N > 0) qm = mtab[sim.mat_e[c] * S + kCoefQM] != 0.0;
    int rb, re;
    record_range(sim, c, rb, re);
    record_fields(sim, c, n1, e, c <= nx - 2 ? hh[c] * sim.h_scale : 0.0, qm, rb, re);
  }
  if (!isfinite(e)) atomicOr(sim.status, kStatusNonFinite);
}

// Launch (per_cu null) or occupancy query (resident tiles per compute unit
// into *per_cu) of one tile shape.  A launch of several chunks needs every
// tile resident at once for the neighbour flags to make progress: the caller
// checks the tile count against the occupancy (and a tile that waits too long
// gives up, so a launch that does not fit ends with an error, not a hang).
template <int N, typename R, int B, int L, bool VC, bool ST, bool P, bool CY, bool BK>
hipError_t launch_shape(const DevSim *sims, const DevTile *tiles, int n_tiles, int64_t n0, int parity, int halo,
                        int k, const ChunkSync &cs, int *per_cu, hipStream_t st) {
  if constexpr (VC && !regs_fit<N, R, B, L>()) {
    // register coefficients are not built for this shape: the same arithmetic
    // with scalar coefficient loads
    return launch_shape<N, R, B, L, false, ST, P, CY, BK>(sims, tiles, n_tiles, n0, parity, halo, k, cs, per_cu, st);
  } else if constexpr (shape_fits<N, R, B, L>() && (!ST || (L == 1 && N >= 2 && (!VC || (N == 3 && B == 256)))) &&
                       (!CY || N >= 2)) {
    auto kern = k_blocked<N, R, B, L, VC, ST, P, CY, BK>;
    if (per_cu) return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, kern, B * L, 0);
    kern<<<n_tiles, B * L, 0, st>>>(sims, tiles, n0, parity, halo, k, cs);
    return hipGetLastError();
  } else {
    return hipErrorInvalidValue;
  }
}

template <int N, typename R, int L, bool VC, bool ST, bool P, bool CY, bool BK>
hipError_t launch_blocked_b(int block, const DevSim *sims, const DevTile *tiles, int n_tiles, int64_t n0,
                            int parity, int halo, int k, const ChunkSync &cs, int *per_cu, hipStream_t st) {
  switch (block) {
    case 64: return launch_shape<N, R, 64, L, VC, ST, P, CY, BK>(sims, tiles, n_tiles, n0, parity, halo, k, cs, per_cu, st);
    case 128: return launch_shape<N, R, 128, L, VC, ST, P, CY, BK>(sims, tiles, n_tiles, n0, parity, halo, k, cs, per_cu, st);
    case 192: return launch_shape<N, R, 192, L, VC, ST, P, CY, BK>(sims, tiles, n_tiles, n0, parity, halo, k, cs, per_cu, st);
    case 256: return launch_shape<N, R, 256, L, VC, ST, P, CY, BK>(sims, tiles, n_tiles, n0, parity, halo, k, cs, per_cu, st);
    case 512: return launch_shape<N, R, 512, L, VC, ST, P, CY, BK>(sims, tiles, n_tiles, n0, parity, halo, k, cs, per_cu, st);
  }
  return hipErrorInvalidValue;
}

// register-resident coefficients are instantiated for the small level counts
// only, split waves for the quantum level counts
template <int N, typename R, bool P, bool CY, bool BK>
hipError_t launch_blocked_nr(int block, int lanes, bool vc, bool strong, const DevSim *sims, const DevTile *tiles,
                             int n_tiles, int64_t n0, int parity, int halo, int k, const ChunkSync &cs, int *per_cu,
                             hipStream_t st) {
  constexpr bool kVC = N == 2 || N == 3;
  // persistent Cayley tiles: one wave per 64 cells only (the other forms
  // report no occupancy, so such runs take one launch per chunk)
  if constexpr (P && CY)
    if (lanes != 1 && !strong) return hipErrorInvalidValue;
  if (strong) {
    // register coefficients for three-level FP32 tiles of 256 cells (the
    // strong step's field iteration otherwise waits on scalar coefficient loads)
    if constexpr (N == 3 && sizeof(R) == 4)
      if (vc && block == 256)
        return launch_shape<N, R, 256, 1, true, true, P, CY, BK>(sims, tiles, n_tiles, n0, parity, halo, k, cs, per_cu, st);
    if constexpr (N >= 2)
      return launch_blocked_b<N, R, 1, false, true, P, CY, BK>(block, sims, tiles, n_tiles, n0, parity, halo, k, cs, per_cu, st);
    return hipErrorInvalidValue;
  }
  switch (lanes) {
    case 1:
      if constexpr (kVC)
        if (vc) return launch_blocked_b<N, R, 1, kVC, false, P, CY, BK>(block, sims, tiles, n_tiles, n0, parity, halo, k, cs, per_cu, st);
      return launch_blocked_b<N, R, 1, false, false, P, CY, BK>(block, sims, tiles, n_tiles, n0, parity, halo, k, cs, per_cu, st);
    case 2:
    case 4:
      if constexpr (N >= 2) {
        if (lanes == 2) {
          if constexpr (kVC)
            if (vc)
              return launch_blocked_b<N, R, 2, kVC, false, P, CY, BK>(block, sims, tiles, n_tiles, n0, parity, halo, k, cs, per_cu, st);
          return launch_blocked_b<N, R, 2, false, false, P, CY, BK>(block, sims, tiles, n_tiles, n0, parity, halo, k, cs, per_cu, st);
        }
        if constexpr (kVC)
          if (vc) return launch_blocked_b<N, R, 4, kVC, false, P, CY, BK>(block, sims, tiles, n_tiles, n0, parity, halo, k, cs, per_cu, st);
        return launch_blocked_b<N, R, 4, false, false, P, CY, BK>(block, sims, tiles, n_tiles, n0, parity, halo, k, cs, per_cu, st);
      }
      break;
    case 8:  // 64-cell tiles of the large density updates only
      if constexpr (N >= 4)
        return launch_blocked_b<N, R, 8, false, false, P, CY, BK>(block, sims, tiles, n_tiles, n0, parity, halo, k, cs, per_cu, st);
      break;
  }
  return hipErrorInvalidValue;
}

// seven and eight levels: one wave per 64 cells on tiles of 128 or 256 cells,
// weak coupling and the exact field step (a cell's state and increments, 90
// and 119 numbers, fill most of a wave's registers; the host refuses the
// other forms at these level counts)
template <int N, typename R, bool P, bool BK>
hipError_t launch_blocked_big(int block, int lanes, bool strong, const DevSim *sims, const DevTile *tiles, int n_tiles,
                              int64_t n0, int parity, int halo, int k, const ChunkSync &cs, int *per_cu,
                              hipStream_t st) {
  if (strong || lanes != 1) return hipErrorInvalidValue;
  switch (block) {
    case 128: return launch_shape<N, R, 128, 1, false, false, P, false, BK>(sims, tiles, n_tiles, n0, parity, halo, k, cs, per_cu, st);
    case 256: return launch_shape<N, R, 256, 1, false, false, P, false, BK>(sims, tiles, n_tiles, n0, parity, halo, k, cs, per_cu, st);
  }
  return hipErrorInvalidValue;
}

template <typename R, bool P, bool CY, bool BK>
hipError_t launch_blocked_r(int levels, int block, int lanes, bool vc, bool strong, const DevSim *sims,
                            const DevTile *tiles, int n_tiles, int64_t n0, int parity, int halo, int k,
                            const ChunkSync &cs, int *per_cu, hipStream_t st) {
  switch (levels) {
#define MB_LEVELS_CASE(n)                                                                                       \
  case n:                                                                                                         \
    return launch_blocked_nr<n, R, P, CY, BK>(block, lanes, vc, strong, sims, tiles, n_tiles, n0, parity, halo, k, cs, per_cu, \
                                   st);
    case 0:
      if constexpr (!BK)
        return launch_blocked_nr<0, R, P, CY, false>(block, lanes, vc, strong, sims, tiles, n_tiles, n0, parity, halo, k,
                                                     cs, per_cu, st);
      break;
    MB_LEVELS_CASE(2)
    MB_LEVELS_CASE(3)
    MB_LEVELS_CASE(4)
    MB_LEVELS_CASE(5)
    MB_LEVELS_CASE(6)
#undef MB_LEVELS_CASE
    case 7:
      if constexpr (!CY)
        return launch_blocked_big<7, R, P, BK>(block, lanes, strong, sims, tiles, n_tiles, n0, parity, halo, k, cs, per_cu, st);
      break;
    case 8:
      if constexpr (!CY)
        return launch_blocked_big<8, R, P, BK>(block, lanes, strong, sims, tiles, n_tiles, n0, parity, halo, k, cs, per_cu, st);
      break;
  }
  return hipErrorInvalidValue;
}

template <int N, typename R>
bool fits_n(int block, int lanes) {
  auto f = [&](auto lc) {
    constexpr int Lc = decltype(lc)::value;
    switch (block) {
      case 64: return shape_fits<N, R, 64, Lc>();
      case 128: return shape_fits<N, R, 128, Lc>();
      case 192: return shape_fits<N, R, 192, Lc>();
      case 256: return shape_fits<N, R, 256, Lc>();
      case 512: return shape_fits<N, R, 512, Lc>();
    }
    return false;
  };
  switch (lanes) {
    case 1: return f(std::integral_constant<int, 1>());
    case 2: return f(std::integral_constant<int, 2>());
    case 4: return f(std::integral_constant<int, 4>());
    case 8: return N >= 4 && f(std::integral_constant<int, 8>());
  }
  return false;
}

template <int N, typename R>
bool regs_n(int block, int lanes) {
  switch (block) {
    case 64: return lanes == 1 ? regs_fit<N, R, 64, 1>() : regs_fit<N, R, 64, 2>();
    case 128: return lanes == 1 ? regs_fit<N, R, 128, 1>() : regs_fit<N, R, 128, 2>();
    case 192: return lanes == 1 ? regs_fit<N, R, 192, 1>() : regs_fit<N, R, 192, 2>();
    case 256: return lanes == 1 ? regs_fit<N, R, 256, 1>() : regs_fit<N, R, 256, 2>();
    case 512: return lanes == 1 ? regs_fit<N, R, 512, 1>() : regs_fit<N, R, 512, 2>();
  }
  return false;
}

template <typename R>
bool fits_r(int levels, int block, int lanes) {
  switch (levels) {
    case 0: return fits_n<0, R>(block, lanes);
    case 2: return fits_n<2, R>(block, lanes);
    case 3: return fits_n<3, R>(block, lanes);
    case 4: return fits_n<4, R>(block, lanes);
    case 5: return fits_n<5, R>(block, lanes);
    case 6: return fits_n<6, R>(block, lanes);
    case 7: return (block == 128 || block == 256) && lanes == 1 && fits_n<7, R>(block, 1);
    case 8: return (block == 128 || block == 256) && lanes == 1 && fits_n<8, R>(block, 1);
  }
  return false;
}

// Work-queue persistent launch of a two- and a three-level tile group (the
// batched parameter sweep): each workgroup takes items (chunk, tile) from the
// counter until none is left and runs one chunk of that tile with the tile
// code of its level count (one wave per 64 cells), so tiles of both level
// counts and of simulations of any length share one launch even when they do
// not all fit on the device at once.
// (waves per SIMD held at 4 for FP32 without register coefficients: the two
// tile bodies together would otherwise take 161 registers, 3 waves, where one
// body alone takes 82 or 121; the 128-register bound costs 100 bytes of spill
// per lane, and the four waves still run a mixed two- and three-level sweep
// 10 % faster than three waves without spill)
template <typename R, int B, bool VC, bool BK>
__global__ void __launch_bounds__(B, (sizeof(R) == 4 && !VC) ? 4 : 2)
    k_queue(QueueArgs qa, int64_t n0, int parity, int halo, int k) {
  union Shared {
    TileShared<2, R, B, 1> two;
    TileShared<3, R, B, 1> three;
  };
  __shared__ Shared sm;
  __shared__ uint32_t item_s;
  const uint32_t per_chunk = uint32_t(qa.n_tiles[0]) + uint32_t(qa.n_tiles[1]);
  const uint32_t total = per_chunk * uint32_t(qa.n_chunks);
  for (;;) {
    __syncthreads();  // the previous item is done with the shared memory
    if (threadIdx.x == 0) item_s = atomicAdd(qa.counter, 1u);
    __syncthreads();
    const uint32_t item = item_s;
    if (item >= total) return;
    const int c = int(item / per_chunk), r = int(item % per_chunk);
    const int64_t nc = n0 + int64_t(c) * k;
    const int par = parity ^ (c & 1);
    if (r < qa.n_tiles[0]) {
      const ChunkSync cs{qa.flags[0], qa.epoch, 1, qa.spin_ticks};
      tile_steps<2, R, B, 1, VC, 0, false, false, false, BK, true>(qa.sims[0], qa.tiles[0], r, c, nc, par, halo, k,
                                                                  cs, sm.two);
    } else {
      const ChunkSync cs{qa.flags[1], qa.epoch, 1, qa.spin_ticks};
      tile_steps<3, R, B, 1, VC, 0, false, false, false, BK, true>(qa.sims[1], qa.tiles[1], r - qa.n_tiles[0], c, nc,
                                                                  par, halo, k, cs, sm.three);
    }
  }
}

// launch (per_cu null) or occupancy query of the work-queue kernel: FP32
// tiles of 128, 192 or 256 cells, FP64 of 128 or 256
template <typename R, bool VC, bool BK>
hipError_t launch_queue_r(int block, int grid, const QueueArgs &qa, int64_t n0, int parity, int halo, int k,
                          int *per_cu, hipStream_t st) {
  auto go = [&](auto kern) -> hipError_t {
    if (per_cu) return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, kern, block, 0);
    kern<<<grid, block, 0, st>>>(qa, n0, parity, halo, k);
    return hipGetLastError();
  };
  switch (block) {
    case 128: return go(k_queue<R, 128, VC, BK>);
    case 192:
      if constexpr (sizeof(R) == 4) return go(k_queue<R, 192, VC, BK>);
      break;
    case 256: return go(k_queue<R, 256, VC, BK>);
  }
  return hipErrorInvalidValue;
}

template <int N, bool BK>
hipError_t launch_plain_n(const DevSim *sims, const DevTile *tiles, int n_tiles, int64_t n0, int parity,
                          hipStream_t st) {
  k_plain_hd<N, BK><<<n_tiles, kPlainBlock, 0, st>>>(sims, tiles, n0, parity);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  k_plain_e<N, BK><<<n_tiles, kPlainBlock, 0, st>>>(sims, tiles, n0, parity);
  return hipGetLastError();
}

}  // namespace

// The kernels are built in eighteen parts so that the library compiles them in
// parallel: for parts 1..16, MB_PART - 1 = id with bit 0 FP64, bit 1
// persistent tiles, bit 2 the Cayley field step, bit 3 the block form; part 2
// also holds the two-launch kernels and the dispatch; parts 17 and 18 the
// work-queue kernels (FP32, FP64); without MB_PART all are built here.
#ifndef MB_PART
#define MB_PART 0
#endif

#define MB_LAUNCH_ARGS                                                                                           \
  int levels, int block, int lanes, bool vc, bool strong, const DevSim *sims, const DevTile *tiles, int n_tiles, \
      int64_t n0, int parity, int halo, int k, const ChunkSync &cs, int *per_cu, hipStream_t st
#define MB_LAUNCH_PASS levels, block, lanes, vc, strong, sims, tiles, n_tiles, n0, parity, halo, k, cs, per_cu, st

hipError_t launch_queue_f32(int block, bool vc, bool bk, int grid, const QueueArgs &qa, int64_t n0, int parity,
                            int halo, int k, int *per_cu, hipStream_t st);
hipError_t launch_queue_f64(int block, bool vc, bool bk, int grid, const QueueArgs &qa, int64_t n0, int parity,
                            int halo, int k, int *per_cu, hipStream_t st);

#define MB_PART_DECLARE(ID) hipError_t launch_part_##ID(MB_LAUNCH_ARGS);
MB_PART_DECLARE(0) MB_PART_DECLARE(1) MB_PART_DECLARE(2) MB_PART_DECLARE(3)
MB_PART_DECLARE(4) MB_PART_DECLARE(5) MB_PART_DECLARE(6) MB_PART_DECLARE(7)
MB_PART_DECLARE(8) MB_PART_DECLARE(9) MB_PART_DECLARE(10) MB_PART_DECLARE(11)
MB_PART_DECLARE(12) MB_PART_DECLARE(13) MB_PART_DECLARE(14) MB_PART_DECLARE(15)
#undef MB_PART_DECLARE

#define MB_PART_DEFINE(ID)                                                                                  \
  hipError_t launch_part_##ID(MB_LAUNCH_ARGS) {                                                             \
    return launch_blocked_r<std::conditional_t<(ID & 1) != 0, double, float>, (ID & 2) != 0, (ID & 4) != 0, \
                            (ID & 8) != 0>(MB_LAUNCH_PASS);                                                 \
  }
#if MB_PART == 0 || MB_PART == 1
MB_PART_DEFINE(0)
#endif
#if MB_PART == 0 || MB_PART == 2
MB_PART_DEFINE(1)
#endif
#if MB_PART == 0 || MB_PART == 3
MB_PART_DEFINE(2)
#endif
#if MB_PART == 0 || MB_PART == 4
MB_PART_DEFINE(3)
#endif
#if MB_PART == 0 || MB_PART == 5
MB_PART_DEFINE(4)
#endif
#if MB_PART == 0 || MB_PART == 6
MB_PART_DEFINE(5)
#endif
#if MB_PART == 0 || MB_PART == 7
MB_PART_DEFINE(6)
#endif
#if MB_PART == 0 || MB_PART == 8
MB_PART_DEFINE(7)
#endif
#if MB_PART == 0 || MB_PART == 9
MB_PART_DEFINE(8)
#endif
#if MB_PART == 0 || MB_PART == 10
MB_PART_DEFINE(9)
#endif
#if MB_PART == 0 || MB_PART == 11
MB_PART_DEFINE(10)
#endif
#if MB_PART == 0 || MB_PART == 12
MB_PART_DEFINE(11)
#endif
#if MB_PART == 0 || MB_PART == 13
MB_PART_DEFINE(12)
#endif
#if MB_PART == 0 || MB_PART == 14
MB_PART_DEFINE(13)
#endif
#if MB_PART == 0 || MB_PART == 15
MB_PART_DEFINE(14)
#endif
#if MB_PART == 0 || MB_PART == 16
MB_PART_DEFINE(15)
#endif
#undef MB_PART_DEFINE

#if MB_PART == 0 || MB_PART == 2
bool block_supported(int block) { return block == 64 || block == 128 || block == 192 || block == 256 || block == 512; }

bool shape_supported(int levels, int precision, int block, int lanes) {
  if (!block_supported(block)) return false;
  return precision == 64 ? fits_r<double>(levels, block, lanes) : fits_r<float>(levels, block, lanes);
}

int plain_block() { return kPlainBlock; }

bool regs_supported(int levels, int precision, int block, int lanes) {
  if (!shape_supported(levels, precision, block, lanes)) return false;
  switch (levels) {
    case 2: return precision == 64 ? regs_n<2, double>(block, lanes) : regs_n<2, float>(block, lanes);
    case 3: return precision == 64 ? regs_n<3, double>(block, lanes) : regs_n<3, float>(block, lanes);
  }
  return false;
}

hipError_t launch_by_id(int id, MB_LAUNCH_ARGS) {
  switch (id) {
    case 0: return launch_part_0(MB_LAUNCH_PASS);
    case 1: return launch_part_1(MB_LAUNCH_PASS);
    case 2: return launch_part_2(MB_LAUNCH_PASS);
    case 3: return launch_part_3(MB_LAUNCH_PASS);
    case 4: return launch_part_4(MB_LAUNCH_PASS);
    case 5: return launch_part_5(MB_LAUNCH_PASS);
    case 6: return launch_part_6(MB_LAUNCH_PASS);
    case 7: return launch_part_7(MB_LAUNCH_PASS);
    case 8: return launch_part_8(MB_LAUNCH_PASS);
    case 9: return launch_part_9(MB_LAUNCH_PASS);
    case 10: return launch_part_10(MB_LAUNCH_PASS);
    case 11: return launch_part_11(MB_LAUNCH_PASS);
    case 12: return launch_part_12(MB_LAUNCH_PASS);
    case 13: return launch_part_13(MB_LAUNCH_PASS);
    case 14: return launch_part_14(MB_LAUNCH_PASS);
    case 15: return launch_part_15(MB_LAUNCH_PASS);
  }
  return hipErrorInvalidValue;
}

int part_id(int precision, bool persistent, bool cayley, bool bk) {
  return (precision == 64 ? 1 : 0) | (persistent ? 2 : 0) | (cayley ? 4 : 0) | (bk ? 8 : 0);
}

hipError_t launch_blocked(int levels, int precision, int block, int lanes, bool vc, bool strong, bool cayley, bool bk,
                          const DevSim *sims, const DevTile *tiles, int n_tiles, int64_t n0, int parity, int halo,
                          int k, const ChunkSync &cs, hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  if (k < 1 || k > halo || k > kMaxChunk || 2 * halo >= block || cs.n_chunks < 1) return hipErrorInvalidValue;
  if (cs.n_chunks > 1 && (!cs.flags || k != halo || 3 * halo > block)) return hipErrorInvalidValue;
  int *per_cu = nullptr;
  return launch_by_id(part_id(precision, cs.n_chunks > 1, cayley, bk && levels > 0), MB_LAUNCH_PASS);
}

// occupancy of the persistent form (the only one that needs every tile resident)
int blocked_tiles_per_cu(int levels, int precision, int block, int lanes, bool vc, bool strong, bool cayley, bool bk) {
  int per_cu_v = 0;
  int *per_cu = &per_cu_v;
  const ChunkSync cs{nullptr, 0u, 2, 0};
  const DevSim *sims = nullptr;
  const DevTile *tiles = nullptr;
  const int n_tiles = 0, parity = 0, halo = 1, k = 1;
  const int64_t n0 = 0;
  hipStream_t st = nullptr;
  const hipError_t e = launch_by_id(part_id(precision, true, cayley, bk && levels > 0), MB_LAUNCH_PASS);
  return e == hipSuccess ? per_cu_v : 0;
}

hipError_t launch_plain(int levels, bool bk, const DevSim *sims, const DevTile *tiles, int n_tiles, int64_t n0,
                        int parity, hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  if (bk) {
    switch (levels) {
      case 2: return launch_plain_n<2, true>(sims, tiles, n_tiles, n0, parity, st);
      case 3: return launch_plain_n<3, true>(sims, tiles, n_tiles, n0, parity, st);
      case 4: return launch_plain_n<4, true>(sims, tiles, n_tiles, n0, parity, st);
      case 5: return launch_plain_n<5, true>(sims, tiles, n_tiles, n0, parity, st);
      case 6: return launch_plain_n<6, true>(sims, tiles, n_tiles, n0, parity, st);
      case 7: return launch_plain_n<7, true>(sims, tiles, n_tiles, n0, parity, st);
      case 8: return launch_plain_n<8, true>(sims, tiles, n_tiles, n0, parity, st);
    }
    return hipErrorInvalidValue;
  }
  switch (levels) {
    case 0: return launch_plain_n<0, false>(sims, tiles, n_tiles, n0, parity, st);
    case 2: return launch_plain_n<2, false>(sims, tiles, n_tiles, n0, parity, st);
    case 3: return launch_plain_n<3, false>(sims, tiles, n_tiles, n0, parity, st);
    case 4: return launch_plain_n<4, false>(sims, tiles, n_tiles, n0, parity, st);
    case 5: return launch_plain_n<5, false>(sims, tiles, n_tiles, n0, parity, st);
    case 6: return launch_plain_n<6, false>(sims, tiles, n_tiles, n0, parity, st);
    case 7: return launch_plain_n<7, false>(sims, tiles, n_tiles, n0, parity, st);
    case 8: return launch_plain_n<8, false>(sims, tiles, n_tiles, n0, parity, st);
  }
  return hipErrorInvalidValue;
}
#endif

// the work-queue kernels: part 17 FP32, part 18 FP64
#if MB_PART == 0 || MB_PART == 17
hipError_t launch_queue_f32(int block, bool vc, bool bk, int grid, const QueueArgs &qa, int64_t n0, int parity,
                            int halo, int k, int *per_cu, hipStream_t st) {
  if (vc)
    return bk ? launch_queue_r<float, true, true>(block, grid, qa, n0, parity, halo, k, per_cu, st)
              : launch_queue_r<float, true, false>(block, grid, qa, n0, parity, halo, k, per_cu, st);
  return bk ? launch_queue_r<float, false, true>(block, grid, qa, n0, parity, halo, k, per_cu, st)
            : launch_queue_r<float, false, false>(block, grid, qa, n0, parity, halo, k, per_cu, st);
}
#endif
#if MB_PART == 0 || MB_PART == 18
hipError_t launch_queue_f64(int block, bool vc, bool bk, int grid, const QueueArgs &qa, int64_t n0, int parity,
                            int halo, int k, int *per_cu, hipStream_t st) {
  if (vc)
    return bk ? launch_queue_r<double, true, true>(block, grid, qa, n0, parity, halo, k, per_cu, st)
              : launch_queue_r<double, true, false>(block, grid, qa, n0, parity, halo, k, per_cu, st);
  return bk ? launch_queue_r<double, false, true>(block, grid, qa, n0, parity, halo, k, per_cu, st)
            : launch_queue_r<double, false, false>(block, grid, qa, n0, parity, halo, k, per_cu, st);
}
#endif
#if MB_PART == 0 || MB_PART == 2
hipError_t launch_queue(int precision, int block, bool vc, bool bk, int grid, const QueueArgs &qa, int64_t n0,
                        int parity, int halo, int k, hipStream_t st) {
  if (grid <= 0 || qa.n_chunks < 1 || k < 1 || k != halo || 3 * halo > block || k > kMaxChunk) return hipErrorInvalidValue;
  return precision == 64 ? launch_queue_f64(block, vc, bk, grid, qa, n0, parity, halo, k, nullptr, st)
                         : launch_queue_f32(block, vc, bk, grid, qa, n0, parity, halo, k, nullptr, st);
}

int queue_tiles_per_cu(int precision, int block, bool vc, bool bk) {
  int per_cu = 0;
  const QueueArgs qa{};
  const hipError_t e = precision == 64 ? launch_queue_f64(block, vc, bk, 0, qa, 0, 0, 1, 1, &per_cu, nullptr)
                                       : launch_queue_f32(block, vc, bk, 0, qa, 0, 0, 1, 1, &per_cu, nullptr);
  return e == hipSuccess ? per_cu : 0;
}
#endif

}  // namespace mb
