// FP64 host plan: grid, FDTD coefficients, Liouvillian and propagators,
// sources and records.  Written from the paper's definitions (Sec. 2-3);
// shares nothing with the CPU oracle used by the tests.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <sstream>

namespace mb {
namespace {

// ---------------------------------------------------------------- small dense helpers

using Mat = std::vector<double>;  // row-major square

Mat matmul(const Mat &a, const Mat &b, int n) {
  Mat c(size_t(n) * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) {
      double aik = a[size_t(i) * n + k];
      if (aik == 0.0) continue;
      for (int j = 0; j < n; ++j) c[size_t(i) * n + j] += aik * b[size_t(k) * n + j];
    }
  return c;
}

double norm1(const Mat &a, int n) {
  double best = 0.0;
  for (int j = 0; j < n; ++j) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += std::fabs(a[size_t(i) * n + j]);
    best = std::max(best, s);
  }
  return best;
}

// e^Z - I by scaling and squaring of a truncated Taylor series (Moler & Van
// Loan, "Nineteen dubious ways", methods 1 and 3), carried without the
// identity: the scaled matrix has 1-norm <= 1/4, where 30 terms of
// Z + Z^2/2! + ... leave a remainder far below double rounding, and each
// squaring (I + E)^2 - I = 2E + E^2 keeps E to its own relative accuracy.
// (Forming e^Z first and subtracting I would leave the small entries of a
// propagator over one time step with an absolute error of an ulp of 1, which
// over many steps drifts a stationary state.)
Mat expm_minus_identity(const Mat &z, int n) {
  double nrm = norm1(z, n);
  int s = 0;
  while (nrm > 0.25) {
    nrm *= 0.5;
    ++s;
  }
  double scale = std::ldexp(1.0, -s);
  Mat zs(z);
  for (double &v : zs) v *= scale;
  Mat result(zs), term(zs);
  for (int k = 2; k <= 30; ++k) {
    term = matmul(term, zs, n);
    double inv = 1.0 / k, tn = 0.0;
    for (double &v : term) {
      v *= inv;
      tn = std::max(tn, std::fabs(v));
    }
    for (size_t q = 0; q < result.size(); ++q) result[q] += term[q];
    if (tn < 1e-300) break;
  }
  for (int q = 0; q < s; ++q) {
    Mat sq = matmul(result, result, n);
    for (size_t i = 0; i < result.size(); ++i) result[i] = 2.0 * result[i] + sq[i];
  }
  return result;
}

// Cyclic Jacobi diagonalisation of a complex Hermitian matrix.  Each
// rotation first removes the phase of a_pq with a diagonal unitary and then
// applies the real symmetric 2 x 2 Jacobi rotation.  Eigenvalues ascending,
// eigenvectors in the columns of v.
void hermitian_eig(int n, std::vector<cd> a, std::vector<double> &lam, std::vector<cd> &v) {
  v.assign(size_t(n) * n, cd(0, 0));
  for (int i = 0; i < n; ++i) v[size_t(i) * n + i] = 1.0;
  auto at = [&](std::vector<cd> &m, int i, int j) -> cd & { return m[size_t(i) * n + j]; };
  double fro = 0.0;
  for (auto &x : a) fro += std::norm(x);
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += std::norm(at(a, p, q));
    if (off <= 1e-34 * fro || off == 0.0) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        cd apq = at(a, p, q);
        double mag = std::abs(apq);
        if (mag == 0.0) continue;
        cd ph = apq / mag;  // e^{i phi}
        double tau = (at(a, q, q).real() - at(a, p, p).real()) / (2.0 * mag);
        double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        // G = D J with D = diag(1, conj(ph)) on (p, q); A <- G^+ A G, V <- V G
        cd gpp = c, gpq = s, gqp = -s * std::conj(ph), gqq = c * std::conj(ph);
        for (int k = 0; k < n; ++k) {  // columns: A G
          cd akp = at(a, k, p), akq = at(a, k, q);
          at(a, k, p) = akp * gpp + akq * gqp;
          at(a, k, q) = akp * gpq + akq * gqq;
          cd vkp = at(v, k, p), vkq = at(v, k, q);
          at(v, k, p) = vkp * gpp + vkq * gqp;
          at(v, k, q) = vkp * gpq + vkq * gqq;
        }
        for (int k = 0; k < n; ++k) {  // rows: G^+ (A G)
          cd apk = at(a, p, k), aqk = at(a, q, k);
          at(a, p, k) = std::conj(gpp) * apk + std::conj(gqp) * aqk;
          at(a, q, k) = std::conj(gpq) * apk + std::conj(gqq) * aqk;
        }
        at(a, p, q) = 0.0;
        at(a, q, p) = 0.0;
      }
  }
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int x, int y) { return at(a, x, x).real() < at(a, y, y).real(); });
  lam.resize(n);
  std::vector<cd> vs(size_t(n) * n);
  for (int k = 0; k < n; ++k) {
    lam[k] = at(a, idx[k], idx[k]).real();
    for (int i = 0; i < n; ++i) vs[size_t(i) * n + k] = at(v, i, idx[k]);
  }
  v = vs;
}

// Smallest eigenvalue of a real symmetric matrix (cyclic Jacobi).
double sym_min_eig(int n, Mat a) {
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = 0; q < n; ++q) {
        tot += a[p * n + q] * a[p * n + q];
        if (p != q) off += a[p * n + q] * a[p * n + q];
      }
    if (off <= 1e-32 * tot || off == 0.0) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = a[p * n + q];
        if (apq == 0.0) continue;
        double tau = (a[q * n + q] - a[p * n + p]) / (2.0 * apq);
        double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int k = 0; k < n; ++k) {
          double akp = a[k * n + p], akq = a[k * n + q];
          a[k * n + p] = c * akp - s * akq;
          a[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          double apk = a[p * n + k], aqk = a[q * n + k];
          a[p * n + k] = c * apk - s * aqk;
          a[q * n + k] = s * apk + c * aqk;
        }
      }
  }
  double m = a[0];
  for (int i = 1; i < n; ++i) m = std::min(m, a[i * n + i]);
  return m;
}

// ---------------------------------------------------------------- quantum description

struct QmFull {
  int n = 0;
  double n3d = 0;
  std::vector<cd> h0, mu;     // N x N row-major
  std::vector<double> rates;  // N x N, rates[i*N+j] = gamma_ij (j -> i)
  std::vector<double> deph;   // packed pairs
  std::vector<std::vector<cd>> ops;  // explicit Lindblad operators (replace rates, deph)
};

// packed index of the pair (i, j), i < j, in column order
inline int pair_index(int i, int j) { return j * (j - 1) / 2 + i; }

std::vector<cd> unpack(int n, const double *diag, const double *off) {
  std::vector<cd> a(size_t(n) * n, cd(0, 0));
  for (int i = 0; i < n; ++i) a[size_t(i) * n + i] = diag ? diag[i] : 0.0;
  for (int j = 1; j < n; ++j)
    for (int i = 0; i < j; ++i) {
      int q = pair_index(i, j);
      cd v = off ? cd(off[2 * q], off[2 * q + 1]) : cd(0, 0);
      a[size_t(i) * n + j] = v;
      a[size_t(j) * n + i] = std::conj(v);
    }
  return a;
}

// a[to[i]][to[j]] <- a[i][j]
std::vector<cd> permute_matrix(int n, const std::vector<cd> &a, const std::vector<int> &to) {
  std::vector<cd> b(a.size());
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) b[size_t(to[i]) * n + to[j]] = a[size_t(i) * n + j];
  return b;
}

// the same quantum description with its levels relabelled (i -> to[i])
void permute_levels(QmFull &q, const std::vector<int> &to) {
  const int n = q.n;
  q.h0 = permute_matrix(n, q.h0, to);
  q.mu = permute_matrix(n, q.mu, to);
  std::vector<double> rates(q.rates.size(), 0.0), deph(q.deph.size(), 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) rates[size_t(to[i]) * n + to[j]] = q.rates[size_t(i) * n + j];
  for (int j = 1; j < n; ++j)
    for (int i = 0; i < j; ++i)
      deph[pair_index(std::min(to[i], to[j]), std::max(to[i], to[j]))] = q.deph[pair_index(i, j)];
  q.rates = rates;
  q.deph = deph;
  for (auto &op : q.ops) op = permute_matrix(n, op, to);
}

int describe(const mb_qm &q, const mb_consts &k, QmFull &out, std::string &err) {
  int n = q.levels;
  if (n < 2 || n > kMaxLevels) {
    err = "level count must be 2..8";
    return MB_ERR_UNSUPPORTED;
  }
  out.n = n;
  out.n3d = q.n3d;
  if (q.two_level) {
    if (n != 2 || q.n_lindblad != 0) {
      err = "two-level form needs levels == 2 and no Lindblad operators";
      return MB_ERR_ARG;
    }
    // Sec. 3.1.1: H0 = hbar w21/2 diag(-1, 1), mu = -e z21 sigma_x
    out.h0 = {cd(-k.hbar * q.omega21 / 2, 0), 0.0, 0.0, cd(k.hbar * q.omega21 / 2, 0)};
    double m = -k.e * q.z21;
    out.mu = {0.0, m, m, 0.0};
    // R = gamma1/2 [[0, 1-w0], [1+w0, 0]], gamma_12,p = gamma2 - gamma1/2
    out.rates = {0.0, q.gamma1 * (1.0 - q.w0) / 2.0, q.gamma1 * (1.0 + q.w0) / 2.0, 0.0};
    out.deph = {q.gamma2 - q.gamma1 / 2.0};
    return MB_OK;
  }
  if (q.n_lindblad < 0 || q.n_lindblad > kMaxLindbladOps || (q.n_lindblad > 0 && !q.lindblad_ops)) {
    err = "n_lindblad must be 0..64, with lindblad_ops when positive";
    return MB_ERR_ARG;
  }
  if (!q.h0_diag || (q.n_lindblad == 0 && (!q.rates || !q.pure_deph))) {
    err = "general quantum description needs h0_diag, and rates and pure_deph or Lindblad operators";
    return MB_ERR_ARG;
  }
  out.h0 = unpack(n, q.h0_diag, q.h0_off);
  out.mu = unpack(n, q.mu_diag, q.mu_off);
  if (q.n_lindblad > 0) {
    // the operators replace the rate form: rates and dephasing stay zero
    out.rates.assign(size_t(n) * n, 0.0);
    out.deph.assign(pair_count(n), 0.0);
    for (int k = 0; k < q.n_lindblad; ++k) {
      std::vector<cd> op(size_t(n) * n);
      for (int e = 0; e < n * n; ++e) {
        const double re = q.lindblad_ops[2 * (size_t(k) * n * n + e)];
        const double im = q.lindblad_ops[2 * (size_t(k) * n * n + e) + 1];
        if (!std::isfinite(re) || !std::isfinite(im)) {
          err = "Lindblad operators must be finite";
          return MB_ERR_ARG;
        }
        op[e] = cd(re, im);
      }
      out.ops.push_back(std::move(op));
    }
    return MB_OK;
  }
  out.rates.assign(q.rates, q.rates + n * n);
  for (int i = 0; i < n; ++i) out.rates[i * n + i] = 0.0;
  out.deph.assign(q.pure_deph, q.pure_deph + pair_count(n));
  for (double r : out.rates)
    if (!(r >= 0.0) || !std::isfinite(r)) {
      err = "scattering rates must be finite and non-negative";
      return MB_ERR_ARG;
    }
  return MB_OK;
}

// L0(rho) = -i/hbar [H0, rho] + D(rho), D in rate form (eq:relax_pop and the
// dephasing law, Sec. 3.1.1) or from explicit Lindblad operators
// (eq:lindbladdiss).  All matrices N x N row-major, original basis.
void apply_free(const QmFull &q, double hbar, const std::vector<cd> &rho, std::vector<cd> &out) {
  int n = q.n;
  out.assign(size_t(n) * n, cd(0, 0));
  const cd mi(0.0, -1.0 / hbar);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      cd acc(0, 0);
      for (int k = 0; k < n; ++k)
        acc += q.h0[size_t(i) * n + k] * rho[size_t(k) * n + j] - rho[size_t(i) * n + k] * q.h0[size_t(k) * n + j];
      out[size_t(i) * n + j] = mi * acc;
    }
  if (!q.ops.empty()) {
    // L rho L^+ - 1/2 (L^+ L rho + rho L^+ L), one operator at a time
    std::vector<cd> lr(size_t(n) * n), ll(size_t(n) * n);
    for (const auto &op : q.ops) {
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
          cd a(0, 0), b(0, 0);
          for (int k = 0; k < n; ++k) {
            a += op[size_t(i) * n + k] * rho[size_t(k) * n + j];               // (L rho)_ij
            b += std::conj(op[size_t(k) * n + i]) * op[size_t(k) * n + j];     // (L^+ L)_ij
          }
          lr[size_t(i) * n + j] = a;
          ll[size_t(i) * n + j] = b;
        }
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
          cd acc(0, 0);
          for (int k = 0; k < n; ++k) {
            acc += lr[size_t(i) * n + k] * std::conj(op[size_t(j) * n + k]);   // (L rho L^+)_ij
            acc -= 0.5 * (ll[size_t(i) * n + k] * rho[size_t(k) * n + j] + rho[size_t(i) * n + k] * ll[size_t(k) * n + j]);
          }
          out[size_t(i) * n + j] += acc;
        }
    }
    return;
  }
  std::vector<double> out_rate(n, 0.0);  // 1/tau_j = sum_{i != j} gamma_ij
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i)
      if (i != j) out_rate[j] += q.rates[i * n + j];
  for (int i = 0; i < n; ++i) {
    cd acc = -out_rate[i] * rho[size_t(i) * n + i];
    for (int j = 0; j < n; ++j)
      if (j != i) acc += q.rates[i * n + j] * rho[size_t(j) * n + j];
    out[size_t(i) * n + i] += acc;
  }
  for (int j = 1; j < n; ++j)
    for (int i = 0; i < j; ++i) {
      double g = 0.5 * (out_rate[i] + out_rate[j]) + q.deph[pair_index(i, j)];
      out[size_t(i) * n + j] -= g * rho[size_t(i) * n + j];
      out[size_t(j) * n + i] -= g * rho[size_t(j) * n + i];
    }
}

// Hermitian matrix from the full real vector v (N^2: populations then pairs)
std::vector<cd> from_real(int n, const std::vector<double> &v) {
  std::vector<cd> a(size_t(n) * n, cd(0, 0));
  for (int k = 0; k < n; ++k) a[size_t(k) * n + k] = v[k];
  for (int j = 1; j < n; ++j)
    for (int i = 0; i < j; ++i) {
      int q = pair_index(i, j);
      cd z(v[n + 2 * q], v[n + 2 * q + 1]);
      a[size_t(i) * n + j] = z;
      a[size_t(j) * n + i] = std::conj(z);
    }
  return a;
}

std::vector<double> to_real(int n, const std::vector<cd> &a) {
  std::vector<double> v(size_t(n) * n, 0.0);
  for (int k = 0; k < n; ++k) v[k] = a[size_t(k) * n + k].real();
  for (int j = 1; j < n; ++j)
    for (int i = 0; i < j; ++i) {
      int q = pair_index(i, j);
      v[n + 2 * q] = a[size_t(i) * n + j].real();
      v[n + 2 * q + 1] = a[size_t(i) * n + j].imag();
    }
  return v;
}

// B = U^+ A U  (to the eigen-basis) or U A U^+ (back)
std::vector<cd> conj_by(int n, const std::vector<cd> &u, const std::vector<cd> &a, bool to_eig) {
  std::vector<cd> t(size_t(n) * n, cd(0, 0)), r(size_t(n) * n, cd(0, 0));
  auto U = [&](int i, int j) { return to_eig ? std::conj(u[size_t(j) * n + i]) : u[size_t(i) * n + j]; };
  auto Ud = [&](int i, int j) { return to_eig ? u[size_t(i) * n + j] : std::conj(u[size_t(j) * n + i]); };
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      cd acc(0, 0);
      for (int k = 0; k < n; ++k) acc += U(i, k) * a[size_t(k) * n + j];
      t[size_t(i) * n + j] = acc;
    }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      cd acc(0, 0);
      for (int k = 0; k < n; ++k) acc += t[size_t(i) * n + k] * Ud(k, j);
      r[size_t(i) * n + j] = acc;
    }
  return r;
}

// x (trace eliminated, M) <-> v (full, N^2): index a < N-1 -> a, else a + 1
inline int full_index(int n, int a) { return a < n - 1 ? a : a + 1; }

std::vector<double> x_to_full(int n, const double *x) {
  int m = state_dim(n);
  std::vector<double> v(size_t(n) * n, 0.0);
  double tr = 0.0;
  for (int a = 0; a < m; ++a) v[full_index(n, a)] = x[a];
  for (int k = 0; k < n - 1; ++k) tr += x[k];
  v[n - 1] = 1.0 - tr;
  return v;
}

// Hermitian rho of the trace-eliminated state x (trace 1)
std::vector<cd> rho_of_x(int n, const double *x) { return from_real(n, x_to_full(n, x)); }

// state coordinates of a traceless Hermitian matrix (the last population is
// minus the sum of the others, so it is dropped)
std::vector<double> x_of_traceless(int n, const std::vector<cd> &a) {
  const int m = state_dim(n);
  std::vector<double> v = to_real(n, a), x(m);
  for (int c = 0; c < m; ++c) x[c] = v[full_index(n, c)];
  return x;
}

// (Re, Im) of the coherences of B = V^+ A V, pairs in packed order
std::vector<double> eig_coherences(int n, const std::vector<cd> &vec, const std::vector<cd> &a) {
  std::vector<cd> b = conj_by(n, vec, a, true);
  std::vector<double> z(size_t(coh_dim(n)));
  for (int kk = 1; kk < n; ++kk)
    for (int j = 0; j < kk; ++j) {
      const int p = pair_index(j, kk);
      z[2 * p] = b[size_t(j) * n + kk].real();
      z[2 * p + 1] = b[size_t(j) * n + kk].imag();
    }
  return z;
}

// The block layout of a material's tables when every entry outside the blocks
// is an exact zero (engine.hpp); otherwise mp.block_form stays false.
void build_block_form(MaterialPlan &mp) {
  const int n = mp.n, m = state_dim(n), kd = coh_dim(n), np = n - 1, pc = pair_count(n);
  auto re = [&](int r) { return np + 2 * r; };  // state row of Re/Im of pair r
  auto im = [&](int r) { return np + 2 * r + 1; };
  auto T = [&](int row, int col) { return mp.tm[size_t(row) * m + col]; };
  auto S = [&](int row, int col) { return mp.sm[size_t(row) * kd + col]; };
  auto A = [&](int row, int col) { return mp.am[size_t(row) * m + col]; };
  bool ok = true;
  for (int q = 0; q < pc && ok; ++q) {
    ok = mp.t0[2 * q + 1] == 0.0;
    for (int a = 0; a < np; ++a) ok = ok && T(2 * q + 1, a) == 0.0 && S(a, 2 * q + 1) == 0.0;
    for (int r = 0; r < pc; ++r)
      ok = ok && T(2 * q, im(r)) == 0.0 && T(2 * q + 1, re(r)) == 0.0 && S(re(r), 2 * q + 1) == 0.0 &&
           S(im(r), 2 * q) == 0.0;
  }
  for (int a = 0; a < m && ok; ++a)
    for (int b = 0; b < m && ok; ++b) {
      const bool pa = a < np, pb = b < np;
      const bool same_pair = !pa && !pb && (a - np) / 2 == (b - np) / 2;
      if (!(pa && pb) && !same_pair) ok = A(a, b) == 0.0;
    }
  for (int a = np; a < m && ok; ++a) ok = mp.bf[a] == 0.0;
  mp.block_form = ok;
  if (!ok) return;
  mp.bfp.assign(mp.bf.begin(), mp.bf.begin() + np);
  mp.ap.assign(size_t(np) * np, 0.0);
  for (int a = 0; a < np; ++a)
    for (int b = 0; b < np; ++b) mp.ap[size_t(a) * np + b] = A(a, b);
  mp.blk.assign(size_t(pc) * 4, 0.0);
  mp.t0r.assign(pc, 0.0);
  mp.tp.assign(size_t(pc) * np, 0.0);
  mp.tr.assign(size_t(pc) * pc, 0.0);
  mp.ti.assign(size_t(pc) * pc, 0.0);
  mp.sp.assign(size_t(np) * pc, 0.0);
  mp.sr.assign(size_t(pc) * pc, 0.0);
  mp.si.assign(size_t(pc) * pc, 0.0);
  for (int r = 0; r < pc; ++r) {
    mp.blk[4 * r + 0] = A(re(r), re(r));
    mp.blk[4 * r + 1] = A(re(r), im(r));
    mp.blk[4 * r + 2] = A(im(r), re(r));
    mp.blk[4 * r + 3] = A(im(r), im(r));
  }
  for (int q = 0; q < pc; ++q) {
    mp.t0r[q] = mp.t0[2 * q];
    for (int a = 0; a < np; ++a) mp.tp[size_t(q) * np + a] = T(2 * q, a);
    for (int r = 0; r < pc; ++r) {
      mp.tr[size_t(q) * pc + r] = T(2 * q, re(r));
      mp.ti[size_t(q) * pc + r] = T(2 * q + 1, im(r));
      mp.sr[size_t(r) * pc + q] = S(re(r), 2 * q);
      mp.si[size_t(r) * pc + q] = S(im(r), 2 * q + 1);
    }
    for (int a = 0; a < np; ++a) mp.sp[size_t(a) * pc + q] = S(a, 2 * q);
  }
}

void build_quantum(MaterialPlan &mp, const QmFull &q, double dt, const mb_consts &k) {
  int n = q.n, m = state_dim(n), nn = n * n, kd = coh_dim(n);
  mp.qm = true;
  mp.n = n;
  mp.n3d = q.n3d;
  hermitian_eig(n, q.mu, mp.lam, mp.vec);
  mp.kappa.resize(n - 1);
  for (int i = 0; i + 1 < n; ++i) mp.kappa[i] = dt * (mp.lam[i] - mp.lam[i + 1]) / k.hbar;
  mp.sigma.resize(n);
  for (int i = 0; i < n; ++i) mp.sigma[i] = dt * mp.lam[i] / k.hbar;
  // full real generator in the operator basis: column a = L0 applied to basis a
  Mat gfull(size_t(nn) * nn, 0.0);
  std::vector<cd> out;
  for (int a = 0; a < nn; ++a) {
    std::vector<double> e(nn, 0.0);
    e[a] = 1.0;
    apply_free(q, k.hbar, from_real(n, e), out);
    std::vector<double> col = to_real(n, out);
    for (int r = 0; r < nn; ++r) gfull[size_t(r) * nn + a] = col[r];
  }
  // trace elimination: rho_{N-1,N-1} = 1 - sum_{k<N-1} x_k
  mp.gen.assign(size_t(m) * m, 0.0);
  mp.gen_off.assign(m, 0.0);
  for (int a = 0; a < m; ++a) {
    int ra = full_index(n, a);
    mp.gen_off[a] = gfull[size_t(ra) * nn + (n - 1)];
    for (int b = 0; b < m; ++b) {
      int cb = full_index(n, b);
      double v = gfull[size_t(ra) * nn + cb];
      if (b < n - 1) v -= gfull[size_t(ra) * nn + (n - 1)];
      mp.gen[size_t(a) * m + b] = v;
    }
  }
  // augmented generator [[G, g], [0, 0]] -> exponentials of dt/2 and dt
  int ma = m + 1;
  Mat z(size_t(ma) * ma, 0.0);
  for (int a = 0; a < m; ++a) {
    for (int b = 0; b < m; ++b) z[size_t(a) * ma + b] = mp.gen[size_t(a) * m + b] * (dt / 2);
    z[size_t(a) * ma + m] = mp.gen_off[a] * (dt / 2);
  }
  // e^{Z} - I for the half step, then the full step (I + E)^2 - I = 2E + E^2;
  // the affine parts are the last columns
  Mat half = expm_minus_identity(z, ma);
  Mat full = matmul(half, half, ma);
  for (size_t i = 0; i < full.size(); ++i) full[i] += 2.0 * half[i];
  mp.ah.assign(size_t(m) * m, 0.0);
  mp.bh.assign(m, 0.0);
  mp.am.assign(size_t(m) * m, 0.0);
  mp.bf.assign(m, 0.0);
  for (int a = 0; a < m; ++a) {
    for (int b = 0; b < m; ++b) {
      mp.ah[size_t(a) * m + b] = half[size_t(a) * ma + b] + (a == b ? 1.0 : 0.0);
      mp.am[size_t(a) * m + b] = full[size_t(a) * ma + b];
    }
    mp.bh[a] = half[size_t(a) * ma + m];
    mp.bf[a] = full[size_t(a) * ma + m];
  }
  // field part: W rho W^+ with W = V diag(e^{i E sigma}) V^+ changes only the
  // eigenbasis coherences z of rho, z_jk -> e^{i theta_jk} z_jk; the step adds
  // the increment V Delta V^+ (Delta: the coherences d = (e^{i theta} - 1) z,
  // zero diagonal), whose state coordinates are sm d.  z = t0 + tm x.
  {
    std::vector<double> zero(m, 0.0);
    mp.t0 = eig_coherences(n, mp.vec, rho_of_x(n, zero.data()));
    mp.tm.assign(size_t(kd) * m, 0.0);
    for (int b = 0; b < m; ++b) {
      std::vector<double> e(m, 0.0);
      e[b] = 1.0;
      std::vector<double> zb = eig_coherences(n, mp.vec, rho_of_x(n, e.data()));
      for (int r = 0; r < kd; ++r) mp.tm[size_t(r) * m + b] = zb[r] - mp.t0[r];
    }
    mp.sm.assign(size_t(m) * kd, 0.0);
    for (int kk = 1; kk < n; ++kk)
      for (int j = 0; j < kk; ++j)
        for (int part = 0; part < 2; ++part) {
          const int r = 2 * pair_index(j, kk) + part;
          const cd v = part == 0 ? cd(1, 0) : cd(0, 1);
          std::vector<cd> delta(size_t(n) * n, cd(0, 0));
          delta[size_t(j) * n + kk] = v;
          delta[size_t(kk) * n + j] = std::conj(v);
          std::vector<double> col = x_of_traceless(n, conj_by(n, mp.vec, delta, false));
          for (int a = 0; a < m; ++a) mp.sm[size_t(a) * kd + r] = col[a];
        }
    mp.bm.assign(size_t(m) * kd, 0.0);
    for (int a = 0; a < m; ++a)
      for (int r = 0; r < kd; ++r) {
        double acc = mp.sm[size_t(a) * kd + r];
        for (int b = 0; b < m; ++b) acc += mp.am[size_t(a) * m + b] * mp.sm[size_t(b) * kd + r];
        mp.bm[size_t(a) * kd + r] = acc;
      }
  }
  // tr{mu X} for a Hermitian X with state coordinates x (trace eliminated):
  // c0 + c . x, c_a = mu_aa - mu_{N-1,N-1}, c_(Re, Im of pair ij) = 2 (Re, Im) mu_ij
  std::vector<double> c(m, 0.0);
  const double mu_last = q.mu[size_t(n - 1) * n + (n - 1)].real();
  for (int a = 0; a < n - 1; ++a) c[a] = q.n3d * (q.mu[size_t(a) * n + a].real() - mu_last);
  for (int j = 1; j < n; ++j)
    for (int i = 0; i < j; ++i) {
      const int p = pair_index(i, j);
      c[n - 1 + 2 * p] = 2.0 * q.n3d * q.mu[size_t(i) * n + j].real();
      c[n + 2 * p] = 2.0 * q.n3d * q.mu[size_t(i) * n + j].imag();
    }
  // p = n3D tr{mu L0(rho^{n+1/2})} = c . xdot, xdot = G (ah y + bh) + g (the
  // derivative is traceless, so c0 drops)
  std::vector<double> cg(m, 0.0);  // c^T G
  for (int b = 0; b < m; ++b)
    for (int a = 0; a < m; ++a) cg[b] += c[a] * mp.gen[size_t(a) * m + b];
  mp.at.assign(m, 0.0);
  for (int b = 0; b < m; ++b)
    for (int a = 0; a < m; ++a) mp.at[b] += cg[a] * mp.ah[size_t(a) * m + b];
  double p0 = 0.0;
  for (int a = 0; a < m; ++a) p0 += cg[a] * mp.bh[a] + c[a] * mp.gen_off[a];
  mp.p0 = p0;
  // strong coupling: (n3D/dt) tr{mu rho} with rho = ah y + bh
  mp.aq.assign(m, 0.0);
  double qc = q.n3d * mu_last;
  for (int a = 0; a < m; ++a) {
    for (int b = 0; b < m; ++b) mp.aq[b] += c[a] * mp.ah[size_t(a) * m + b];
    qc += c[a] * mp.bh[a];
  }
  for (double &v : mp.aq) v /= dt;
  mp.qc = qc / dt;
  // readouts of y = x + sm d folded: the d parts
  auto fold = [&](const std::vector<double> &r) {
    std::vector<double> rs(kd, 0.0);
    for (int t = 0; t < kd; ++t)
      for (int a = 0; a < m; ++a) rs[t] += r[a] * mp.sm[size_t(a) * kd + t];
    return rs;
  };
  mp.as = fold(mp.at);
  mp.aqs = fold(mp.aq);
  build_block_form(mp);
  // complete positivity of the pure dephasing: Gram matrix -1/2 J D J, D_ij = 2 gamma_ij,p
  Mat d(size_t(n) * n, 0.0), jm(size_t(n) * n, 0.0);
  double dmax = 0.0;
  for (int j = 1; j < n; ++j)
    for (int i = 0; i < j; ++i) {
      d[i * n + j] = d[j * n + i] = 2.0 * q.deph[pair_index(i, j)];
      dmax = std::max(dmax, std::fabs(d[i * n + j]));
    }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) jm[i * n + j] = (i == j ? 1.0 : 0.0) - 1.0 / n;
  Mat g = matmul(matmul(jm, d, n), jm, n);
  for (double &v : g) v *= -0.5;
  mp.min_gram_eig = sym_min_eig(n, g) / std::max(dmax, 1e-300);
}

// value of a density quantity for a full real vector v (operator basis)
double quantity_of(const MaterialPlan &mp, int quantity, int i, int j, const std::vector<double> &v) {
  int n = mp.n;
  std::vector<cd> rho = from_real(n, v);
  i = mp.lvl[i];
  j = mp.lvl[j];
  switch (quantity) {
    case MB_REC_POP: return rho[size_t(i) * n + i].real();
    case MB_REC_INV: return (rho[size_t(j) * n + j] - rho[size_t(i) * n + i]).real();
    case MB_REC_RHO_RE: return rho[size_t(i) * n + j].real();
    case MB_REC_RHO_IM: return rho[size_t(i) * n + j].imag();
  }
  return 0.0;
}

// Readout (r0, r, rs) with value = r0 + r . x + rs . d for the state x and the
// field increments d of the step: rho^{n+1/2} = ah y + bh, y = x + sm d.
void build_readout(const MaterialPlan &mp, int quantity, int i, int j, double *out) {
  int n = mp.n, m = state_dim(n), kd = coh_dim(n);
  std::vector<double> zero(m, 0.0);
  double base = quantity_of(mp, quantity, i, j, x_to_full(n, zero.data()));
  std::vector<double> r(m, 0.0);
  for (int a = 0; a < m; ++a) {
    std::vector<double> e(m, 0.0);
    e[a] = 1.0;
    r[a] = quantity_of(mp, quantity, i, j, x_to_full(n, e.data())) - base;
  }
  double r0 = base;
  for (int a = 0; a < m; ++a) r0 += r[a] * mp.bh[a];
  out[0] = r0;
  for (int b = 0; b < m; ++b) {
    double acc = 0.0;
    for (int a = 0; a < m; ++a) acc += r[a] * mp.ah[size_t(a) * m + b];
    out[1 + b] = acc;
  }
  for (int t = 0; t < kd; ++t) {
    double acc = 0.0;
    for (int b = 0; b < m; ++b) acc += out[1 + b] * mp.sm[size_t(b) * kd + t];
    out[1 + m + t] = acc;
  }
}

double source_value(const mb_source &s, double t) {
  double env = 0.0;
  int cnt = std::max(1, s.count);
  for (int q = 0; q < cnt; ++q) {
    double arg = s.width * (t - q * s.period) - s.shift;
    if (s.kind == MB_SRC_SECH)
      env += std::fabs(arg) < 700.0 ? 1.0 / std::cosh(arg) : 0.0;
    else
      env += std::exp(-arg * arg);
  }
  return s.amp * env * std::sin(2.0 * M_PI * s.freq * t + s.phase);
}

// Node of a source at position x (Sec. 3.2 converts positions to integer grid
// indices at set-up): round(x/dx) with halves to the even node; -1 outside the
// grid.  A single-point device (nx = 1) has its one node at x = 0.
int64_t source_node(double x, double dx, int64_t nx) {
  if (!std::isfinite(x)) return -1;
  if (nx == 1) return x == 0.0 ? 0 : -1;
  const double q = x / dx;
  if (!(q > -1.0 && q < double(nx))) return -1;
  double r = std::floor(q);
  const double f = q - r;
  if (f > 0.5 || (f == 0.5 && std::fmod(r, 2.0) != 0.0)) r += 1.0;
  return r >= 0.0 && r <= double(nx - 1) ? int64_t(r) : -1;
}

int region_material(const mb_device_desc *dev, double x, double dx, std::string &err) {
  for (int r = 0; r < dev->n_regions; ++r)
    if (dev->regions[r].x_start <= x && x < dev->regions[r].x_end) return dev->regions[r].material;
  for (int r = 0; r < dev->n_regions; ++r)
    if (dev->regions[r].x_start <= x && x <= dev->regions[r].x_end) return dev->regions[r].material;
  int best = -1;
  double end = -1e300;
  for (int r = 0; r < dev->n_regions; ++r)
    if (dev->regions[r].x_end > end) {
      end = dev->regions[r].x_end;
      best = r;
    }
  if (best >= 0 && x > end && x <= end + 0.5 * dx) return dev->regions[best].material;
  std::ostringstream os;
  os << "grid point x=" << x << " lies in no region";
  err = os.str();
  return -1;
}

}  // namespace

bool solve_linear(int n, std::vector<double> a, std::vector<double> &b) {
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(a[size_t(r) * n + c]) > std::fabs(a[size_t(piv) * n + c])) piv = r;
    if (a[size_t(piv) * n + c] == 0.0) return false;
    if (piv != c) {
      for (int k = 0; k < n; ++k) std::swap(a[size_t(c) * n + k], a[size_t(piv) * n + k]);
      std::swap(b[c], b[piv]);
    }
    for (int r = c + 1; r < n; ++r) {
      double f = a[size_t(r) * n + c] / a[size_t(c) * n + c];
      if (f == 0.0) continue;
      for (int k = c; k < n; ++k) a[size_t(r) * n + k] -= f * a[size_t(c) * n + k];
      b[r] -= f * b[c];
    }
  }
  for (int c = n - 1; c >= 0; --c) {
    double acc = b[c];
    for (int k = c + 1; k < n; ++k) acc -= a[size_t(c) * n + k] * b[k];
    b[c] = acc / a[size_t(c) * n + c];
  }
  return true;
}

void state_to_rho(const MaterialPlan &mp, const double *sigma, cd *rho) {
  int n = mp.n, m = state_dim(n);
  std::vector<double> rhs(m);
  for (int a = 0; a < m; ++a) rhs[a] = sigma[a] - mp.bh[a];
  solve_linear(m, mp.ah, rhs);
  std::vector<cd> r = rho_of_x(n, rhs.data());
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) rho[size_t(i) * n + j] = r[size_t(mp.lvl[i]) * n + mp.lvl[j]];
}

int build_plan(const mb_device_desc *dev, const mb_scenario_desc *scen, SimPlan &plan,
               std::string &err) {
  if (!dev || !scen) {
    err = "null description";
    return MB_ERR_ARG;
  }
  const mb_consts &k = scen->consts;
  if (!(k.hbar > 0 && k.c0 > 0 && k.mu0 > 0 && k.eps0 > 0 && k.e > 0)) {
    err = "physical constants must be positive";
    return MB_ERR_ARG;
  }
  if (scen->nx < 1 || scen->n_steps < 0 || !(scen->dt > 0) || !std::isfinite(scen->dt)) {
    err = "need nx >= 1, n_steps >= 0 and a positive time step";
    return MB_ERR_ARG;
  }
  if (scen->nx == 2) {
    err = "nx must be 1 (single point) or at least 3 (two edge nodes and an interior)";
    return MB_ERR_ARG;
  }
  if (scen->nx >= (int64_t(1) << 26) || scen->n_steps >= (int64_t(1) << 31) - 1) {
    err = "grid or step count too large for 32-bit indexing";
    return MB_ERR_ARG;
  }
  if (scen->precision != 64 && scen->precision != 32) {
    err = "precision must be 64 or 32";
    return MB_ERR_ARG;
  }
  if (scen->variant < MB_VARIANT_AUTO || scen->variant > MB_VARIANT_BLOCKED_REGS) {
    err = "unknown variant";
    return MB_ERR_ARG;
  }
  if (scen->lanes != 0 && scen->lanes != 1 && scen->lanes != 2 && scen->lanes != 4 && scen->lanes != 8) {
    err = "lanes must be 0, 1, 2, 4 or 8";
    return MB_ERR_ARG;
  }
  if (scen->coupling != MB_COUPLING_WEAK && scen->coupling != MB_COUPLING_STRONG) {
    err = "coupling must be MB_COUPLING_WEAK or MB_COUPLING_STRONG";
    return MB_ERR_ARG;
  }
  if (scen->field_step != MB_FIELD_EXACT && scen->field_step != MB_FIELD_CAYLEY) {
    err = "field_step must be MB_FIELD_EXACT or MB_FIELD_CAYLEY";
    return MB_ERR_ARG;
  }
  if (scen->coupling == MB_COUPLING_STRONG && scen->variant == MB_VARIANT_PLAIN) {
    err = "strong coupling runs on the blocked variant";
    return MB_ERR_UNSUPPORTED;
  }
  if (scen->variant == MB_VARIANT_PLAIN && scen->precision != 64) {
    err = "the plain variant runs in FP64 only";
    return MB_ERR_UNSUPPORTED;
  }
  if (dev->n_materials < 1 || dev->n_materials > 255 || !dev->materials || dev->n_regions < 1 ||
      !dev->regions) {
    err = "need 1..255 materials and at least one region";
    return MB_ERR_ARG;
  }
  for (double r : {dev->refl_left, dev->refl_right})
    if (!(r >= 0.0 && r <= 1.0)) {
      err = "reflectivities must lie in [0, 1]";
      return MB_ERR_ARG;
    }
  for (int r = 0; r < dev->n_regions; ++r)
    if (dev->regions[r].material < 0 || dev->regions[r].material >= dev->n_materials) {
      err = "region refers to a missing material";
      return MB_ERR_ARG;
    }
  plan = SimPlan();
  plan.nx = scen->nx;
  plan.n_steps = scen->n_steps;
  plan.dt = scen->dt;
  plan.precision = scen->precision;
  plan.variant = scen->variant;
  plan.block = scen->block;
  plan.depth = scen->depth;
  plan.lanes = scen->lanes;
  plan.coupling = scen->coupling;
  plan.field_step = scen->field_step;
  plan.dx = scen->nx > 1 ? dev->length / double(scen->nx - 1) : 0.0;
  if (scen->nx > 1 && !(plan.dx > 0)) {
    err = "device length must be positive";
    return MB_ERR_ARG;
  }
  const int64_t nx = plan.nx;
  plan.mat_e.resize(nx);
  plan.mat_h.resize(nx, 0);
  for (int64_t c = 0; c < nx; ++c) {
    int m = region_material(dev, double(c) * plan.dx, plan.dx, err);
    if (m < 0) return MB_ERR_ARG;
    plan.mat_e[c] = uint8_t(m);
    if (c + 1 < nx) {
      int mh = region_material(dev, (double(c) + 0.5) * plan.dx, plan.dx, err);
      if (mh < 0) return MB_ERR_ARG;
      plan.mat_h[c] = uint8_t(mh);
    }
  }
  // FDTD coefficients per material (Sec. 3.2) and the Courant check
  plan.mats.resize(dev->n_materials);
  double c_max = 0.0;
  int levels = 0;
  std::vector<QmFull> qms(dev->n_materials);
  for (int i = 0; i < dev->n_materials; ++i) {
    const mb_material &mt = dev->materials[i];
    MaterialPlan &mp = plan.mats[i];
    if (!(mt.eps_r > 0 && mt.mu_r > 0 && mt.alpha0 >= 0 && std::isfinite(mt.overlap))) {
      err = "material needs eps_r > 0, mu_r > 0, alpha0 >= 0";
      return MB_ERR_ARG;
    }
    mp.eps_r = mt.eps_r;
    mp.mu_r = mt.mu_r;
    mp.alpha0 = mt.alpha0;
    mp.overlap = mt.overlap;
    double eps = k.eps0 * mt.eps_r, mu = k.mu0 * mt.mu_r;
    const double eta0 = std::sqrt(k.mu0 / k.eps0);
    double sigma = 2.0 * mt.alpha0 * std::sqrt(eps / mu);
    double q = plan.dt * sigma / (2.0 * eps);
    double bb = (plan.dt / eps) / (1.0 + q);
    mp.ca = (1.0 - q) / (1.0 + q);
    mp.cbg = bb * mt.overlap;
    // E and eta0 H: the curl coefficients become c0 dt/(eps_r dx (1 + q)) and
    // c0 dt/(mu_r dx), exact in FP32 for Courant numbers such as 1/2 (with the
    // SI coefficients their FP32 roundings change the wave speed by ~1e-8,
    // a phase error of ~1e-4 after 1e4 cells of propagation)
    mp.cbd = nx > 1 ? bb / (plan.dx * eta0) : 0.0;
    mp.ch = nx > 1 ? plan.dt * eta0 / (plan.dx * mu) : 0.0;
    mp.c_light = 1.0 / std::sqrt(eps * mu);
    c_max = std::max(c_max, mp.c_light);
    if (mt.qm) {
      int rc = describe(*mt.qm, k, qms[i], err);
      if (rc < 0) return rc;
      if (levels && levels != qms[i].n) {
        err = "all quantum materials of one device must have the same level count";
        return MB_ERR_UNSUPPORTED;
      }
      levels = qms[i].n;
    }
  }
  if (nx > 1 && c_max * plan.dt > plan.dx * (1.0 + 1e-12)) {
    err = "time step exceeds the Courant limit dx / c_max";
    return MB_ERR_CFL;
  }
  if (levels >= 7 && scen->variant != MB_VARIANT_PLAIN &&
      (scen->coupling == MB_COUPLING_STRONG || scen->field_step == MB_FIELD_CAYLEY)) {
    err = "7 and 8 levels run with weak coupling and the exact field step";
    return MB_ERR_UNSUPPORTED;
  }
  plan.n = levels;
  plan.m = levels ? state_dim(levels) : 0;
  std::vector<int> lvl;
  if (levels) {
    if (!scen->rho_diag) {
      err = "initial density matrix missing";
      return MB_ERR_ARG;
    }
    // the most populated initial level (the last of equals) goes last
    int top = 0;
    for (int i = 1; i < levels; ++i)
      if (scen->rho_diag[i] >= scen->rho_diag[top]) top = i;
    for (int i = 0, at = 0; i < levels; ++i) lvl.push_back(i == top ? levels - 1 : at++);
  }
  // the block form wherever the tables allow it (MB_BLOCK_FORM=0: never)
  const char *bf_env = std::getenv("MB_BLOCK_FORM");
  plan.block_form = levels > 0 && !(bf_env && bf_env[0] == '0');
  for (int i = 0; i < dev->n_materials; ++i)
    if (dev->materials[i].qm) {
      permute_levels(qms[i], lvl);
      plan.mats[i].lvl = lvl;
      build_quantum(plan.mats[i], qms[i], plan.dt, k);
      plan.block_form = plan.block_form && plan.mats[i].block_form;
      if (plan.mats[i].min_gram_eig < -1e-9) plan.warn = MB_WARN_NOT_CP;
    }
  // edges (Sec. 2.1): R = 1 perfect conductor, R = 0 first-order Mur, 0 < R < 1 a
  // resistive load Z_L = eta (1 - sqrt R)/(1 + sqrt R) on the edge node's half cell,
  // amplitude reflection -sqrt R; Ampere's law over the half cell with the load
  // current at t_{n+1/2} gives E' = g E +- d H_inner, a = dt/(eps dx Z_L),
  // g = (1 - a)/(1 + a), d = 2 dt/(eps dx)/(1 + a)
  auto edge_kind = [](double r) { return r == 1.0 ? 0 : r == 0.0 ? 1 : 2; };
  plan.h_scale = 1.0 / std::sqrt(k.mu0 / k.eps0);
  plan.edge_l = edge_kind(dev->refl_left);
  plan.edge_r = edge_kind(dev->refl_right);
  if (nx > 1) {
    double cl = plan.mats[plan.mat_e[0]].c_light, cr = plan.mats[plan.mat_e[nx - 1]].c_light;
    plan.kap_l = (cl * plan.dt - plan.dx) / (cl * plan.dt + plan.dx);
    plan.kap_r = (cr * plan.dt - plan.dx) / (cr * plan.dt + plan.dx);
    auto load = [&](const MaterialPlan &mp, double r, double &g, double &d) {
      const double eps = k.eps0 * mp.eps_r, mu = k.mu0 * mp.mu_r;
      const double sr = std::sqrt(r), zl = std::sqrt(mu / eps) * (1.0 - sr) / (1.0 + sr);
      const double a = plan.dt / (eps * plan.dx * zl);
      g = (1.0 - a) / (1.0 + a);
      d = 2.0 * plan.dt / (eps * plan.dx) / (1.0 + a) / std::sqrt(k.mu0 / k.eps0);  // acts on eta0 H
    };
    if (plan.edge_l == 2) load(plan.mats[plan.mat_e[0]], dev->refl_left, plan.load_g_l, plan.load_d_l);
    if (plan.edge_r == 2) load(plan.mats[plan.mat_e[nx - 1]], dev->refl_right, plan.load_g_r, plan.load_d_r);
  }
  // sources: FP64 tables s(n dt), n = 0..n_steps
  if (scen->n_sources < 0 || (scen->n_sources > 0 && !scen->sources)) {
    err = "bad source list";
    return MB_ERR_ARG;
  }
  for (int s = 0; s < scen->n_sources; ++s) {
    const mb_source &src = scen->sources[s];
    const int64_t cell = source_node(src.x, plan.dx, nx);
    if (cell < 0 || (src.kind != MB_SRC_SECH && src.kind != MB_SRC_GAUSS && src.kind != MB_SRC_TABLE)) {
      err = "source outside the grid or of unknown kind";
      return MB_ERR_ARG;
    }
    if (src.kind == MB_SRC_TABLE && (src.table_len < 0 || (src.table_len > 0 && !src.table))) {
      err = "table source needs table_len >= 0 values";
      return MB_ERR_ARG;
    }
    SourcePlan sp;
    sp.cell = cell;
    sp.hard = src.hard ? 1 : 0;
    sp.table.resize(plan.n_steps + 1);
    for (int64_t t = 0; t <= plan.n_steps; ++t)
      sp.table[t] = src.kind == MB_SRC_TABLE ? (t < src.table_len ? src.table[t] : 0.0)
                                             : source_value(src, double(t) * plan.dt);
    for (double v : sp.table)
      if (!std::isfinite(v)) {
        err = "source values must be finite";
        return MB_ERR_ARG;
      }
    plan.sources.push_back(std::move(sp));
  }
  // records
  if (scen->n_records < 0 || (scen->n_records > 0 && !scen->records)) {
    err = "bad record list";
    return MB_ERR_ARG;
  }
  for (int r = 0; r < scen->n_records; ++r) {
    const mb_record &rc = scen->records[r];
    RecordPlan rp;
    rp.quantity = rc.quantity;
    rp.i = rc.i;
    rp.j = rc.j;
    rp.cell = rc.cell;
    rp.interval = rc.interval;
    if (rc.quantity < MB_REC_E || rc.quantity > MB_REC_RHO_IM || rc.interval < 1 || rc.cell < -1 ||
        rc.cell >= nx) {
      err = "record with unknown quantity, bad interval or cell";
      return MB_ERR_ARG;
    }
    bool dens = rc.quantity >= MB_REC_POP;
    if (dens && (levels == 0 || rc.i < 0 || rc.j < 0 || rc.i >= levels || rc.j >= levels)) {
      err = "density record needs quantum cells and levels in range";
      return MB_ERR_ARG;
    }
    if ((rc.quantity == MB_REC_RHO_RE || rc.quantity == MB_REC_RHO_IM) && rc.i == rc.j &&
        rc.quantity == MB_REC_RHO_IM) {
      // Im of a diagonal element is identically zero; allowed
    }
    rp.width = rc.cell < 0 ? nx : 1;
    rp.n_samples = plan.n_steps / rp.interval;
    if (dens) {
      const int rl = plan.m + 1 + coh_dim(levels);
      rp.readout.assign(size_t(dev->n_materials) * rl, 0.0);
      for (int i = 0; i < dev->n_materials; ++i)
        if (plan.mats[i].qm) build_readout(plan.mats[i], rc.quantity, rc.i, rc.j, &rp.readout[size_t(i) * rl]);
    }
    plan.records.push_back(std::move(rp));
  }
  // initial state: E^0 (edges, hard sources at t = 0), sigma_0 = e^{L0 dt/2} rho_init
  plan.e0.assign(nx, 0.0);
  if (!std::isfinite(scen->e_const) || !std::isfinite(scen->e_noise)) {
    err = "e_const and e_noise must be finite";
    return MB_ERR_ARG;
  }
  if (scen->e_init) {
    for (int64_t c = 0; c < nx; ++c) plan.e0[c] = scen->e_init[c];
  } else {
    // SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): a Weyl sequence with
    // increment 0x9E3779B97F4A7C15 passed through a 64-bit finaliser
    uint64_t state = scen->e_seed;
    for (int64_t c = 0; c < nx; ++c) {
      double v = scen->e_const;
      if (scen->e_noise != 0.0) {
        state += 0x9E3779B97F4A7C15ull;
        uint64_t z = state;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        const double u = double(z >> 11) * 0x1.0p-53;
        v += scen->e_noise * (2.0 * u - 1.0);
      }
      plan.e0[c] = v;
    }
  }
  if (nx > 1) {
    if (plan.edge_l == 0) plan.e0[0] = 0.0;
    if (plan.edge_r == 0) plan.e0[nx - 1] = 0.0;
  }
  for (auto &sp : plan.sources)
    if (sp.hard) plan.e0[sp.cell] = sp.table[0];
  if (levels) {
    if (!scen->rho_diag) {
      err = "initial density matrix missing";
      return MB_ERR_ARG;
    }
    int n = levels, m = plan.m;
    std::vector<cd> rho0 = permute_matrix(n, unpack(n, scen->rho_diag, scen->rho_off), lvl);
    plan.x0.assign(size_t(m) * nx, 0.0);
    plan.q0.assign(nx, 0.0);
    for (int i = 0; i < dev->n_materials; ++i) {
      const MaterialPlan &mp = plan.mats[i];
      if (!mp.qm) continue;
      std::vector<double> v = to_real(n, rho0);
      std::vector<double> x(m);
      for (int a = 0; a < m; ++a) x[a] = v[full_index(n, a)];
      std::vector<double> sig(m);
      for (int a = 0; a < m; ++a) {
        double acc = mp.bh[a];
        for (int b = 0; b < m; ++b) acc += mp.ah[size_t(a) * m + b] * x[b];
        sig[a] = acc;
      }
      // (n3D/dt) tr{mu rho^0}
      double q = 0.0;
      for (int a = 0; a < n; ++a) q += (qms[i].mu[size_t(a) * n + a] * rho0[size_t(a) * n + a]).real();
      for (int jj = 1; jj < n; ++jj)
        for (int ii = 0; ii < jj; ++ii) q += 2.0 * (qms[i].mu[size_t(jj) * n + ii] * rho0[size_t(ii) * n + jj]).real();
      q *= mp.n3d / plan.dt;
      for (int64_t c = 0; c < nx; ++c)
        if (plan.mat_e[c] == i) {
          for (int a = 0; a < m; ++a) plan.x0[size_t(a) * nx + c] = sig[a];
          plan.q0[c] = q;
        }
    }
  }
  for (double v : plan.e0)
    if (!std::isfinite(v)) {
      err = "non-finite initial field";
      return MB_ERR_ARG;
    }
  return plan.warn;
}

}  // namespace mb
