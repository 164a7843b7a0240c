// Host-side FP64 plan of one simulation: everything the kernels need, computed
// once per simulation before the first step.
#pragma once

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "mb.h"

namespace mb {

using cd = std::complex<double>;

constexpr int kMaxLevels = 8;
constexpr int kMaxLindbladOps = 64;

// Real parametrisation of an N x N Hermitian density matrix in the basis the
// operators are given in: populations 0..N-2 (the last one is 1 - sum, trace
// elimination), then (Re, Im) of each upper pair in packed order
// (1,2),(1,3),(2,3),...  Dimension M = N*N - 1.  The field part works on the
// (Re, Im) coordinates of the coherences in the dipole eigenbasis (K = N*(N-1)
// reals, same pair order).
inline int state_dim(int n) { return n * n - 1; }
inline int pair_count(int n) { return n * (n - 1) / 2; }
inline int coh_dim(int n) { return n * (n - 1); }

struct MaterialPlan {
  double eps_r = 1, mu_r = 1, alpha0 = 0, overlap = 1;
  double ca = 1, cbg = 0, cbd = 0, ch = 0;  // a', b' Gamma, b'/dx, c'
  double c_light = 0;
  bool qm = false;
  int n = 0;
  double n3d = 0;
  // the levels in the order the tables use: lvl[i] = position of the caller's
  // level i (the most populated initial level is moved last, where the trace
  // elimination puts it, so that it is never stored: an FP32 state then holds
  // only populations it can resolve relative to their own size)
  std::vector<int> lvl;
  // quantum tables (FP64); states in the operator basis, trace eliminated
  std::vector<double> lam;        // N sorted eigenvalues of mu
  std::vector<cd> vec;            // N x N eigenvectors (columns), row-major
  std::vector<double> kappa;      // N-1: dt (lam_q - lam_{q+1}) / hbar
  std::vector<double> sigma;      // N: dt lam_j / hbar (Cayley field step)
  std::vector<double> gen;        // M x M generator of L0 (x' = G x + g)
  std::vector<double> gen_off;    // M
  std::vector<double> ah, bh;     // e^{L0 dt/2}: x -> ah x + bh
  std::vector<double> am, bf;     // e^{L0 dt} - I and its affine part
  std::vector<double> t0, tm;     // K, K x M: eigenbasis coherences z = t0 + tm x
  std::vector<double> sm;         // M x K: field increment d (eigenbasis) -> state coordinates
  std::vector<double> bm;         // M x K: e^{L0 dt} sm
  std::vector<double> at;         // M: p = at . y + p0, y = x + sm d
  std::vector<double> as;         // K: at sm
  double p0 = 0;
  std::vector<double> aq;         // M: strong coupling, (n3D/dt) tr{mu rho} = aq . y + qc
  std::vector<double> aqs;        // K: aq sm
  double qc = 0;
  // block form (engine.hpp): the tables above have exact zeros outside the
  // population block, the 2 x 2 pair blocks and the real/imaginary split of
  // z and of the increment map (a real dipole operator, H0 diagonal,
  // relaxation in rate form); then the same step in the block layout
  bool block_form = false;
  std::vector<double> bfp, ap, blk, t0r, tp, tr, ti, sp, sr, si;
  double min_gram_eig = 0;        // complete-positivity check of the dephasing rates
};

struct SourcePlan {
  int64_t cell = 0;
  int hard = 1;
  std::vector<double> table;      // s(n dt), n = 0..n_steps
};

struct RecordPlan {
  int quantity = 0, i = 0, j = 0;
  int64_t cell = 0, interval = 1, width = 1, n_samples = 0;
  // density quantities: per material M+1+K doubles: value = r0 + r . x + rs . d
  std::vector<double> readout;
};

struct SimPlan {
  int64_t nx = 0, n_steps = 0;
  double dt = 0, dx = 0;
  int n = 0, m = 0;               // levels (0: no quantum cells) and state dimension
  int precision = 64;
  int variant = MB_VARIANT_AUTO;
  int block = 0, depth = 0, lanes = 0;
  int coupling = MB_COUPLING_WEAK;
  int field_step = MB_FIELD_EXACT;
  bool block_form = false;        // every quantum material in block form
  std::vector<uint8_t> mat_e, mat_h;
  std::vector<MaterialPlan> mats;
  int edge_l = 0, edge_r = 0;     // 0: PEC, 1: Mur, 2: impedance load (0 < R < 1)
  double kap_l = 0, kap_r = 0;    // Mur coefficients
  double load_g_l = 0, load_d_l = 0, load_g_r = 0, load_d_r = 0;  // E' = g E +- d H'_inner
  // E and H' = eta0 H are advanced (eta0 = sqrt(mu0/eps0)); H = h_scale H'
  double h_scale = 1.0;
  std::vector<SourcePlan> sources;
  std::vector<RecordPlan> records;
  std::vector<double> e0;         // nx
  std::vector<double> x0;         // m planes of nx: the running state sigma_0
  std::vector<double> q0;         // strong coupling: (n3D/dt) tr{mu rho^0} per cell
  int warn = MB_OK;
};

// Builds the plan.  Returns MB_OK, MB_WARN_NOT_CP or a negative error with
// a message in err.
int build_plan(const mb_device_desc *dev, const mb_scenario_desc *scen, SimPlan &plan,
               std::string &err);

// Host linear algebra used by the plan (exposed for the state read-back).
bool solve_linear(int n, std::vector<double> a, std::vector<double> &b);

// rho (N x N complex, operator basis) of the running state x of a material:
// rho^{n-1/2} = inverse half-propagator of sigma.
void state_to_rho(const MaterialPlan &mp, const double *sigma, cd *rho);

}  // namespace mb
