// HIP kernels for gfx950: one time step of the 1D Maxwell-Bloch system per
// cell and lane.  State is structure-of-arrays (E, H and the M = N*N - 1
// density parameters as separate planes), coefficients are per material and
// read with wave-uniform addresses, every step of a cell is the same
// arithmetic in the two-launch and in the blocked kernels (explicit fma, no
// contraction), so both produce bit-identical results.
#include <hip/hip_runtime.h>

#include "engine.hpp"
#include "launch.hpp"

namespace mb {
namespace {

__device__ __forceinline__ void sincos_r(double a, double *s, double *c) { sincos(a, s, c); }
__device__ __forceinline__ void sincos_r(float a, float *s, float *c) { sincosf(a, s, c); }

template <int N, typename R>
struct Cell {
  static constexpr int M = mat_m(N);
  static constexpr int MA = M > 0 ? M : 1;

  // y <- Phi_E(y): coherence (j, k), j < k, of the state in the dipole
  // eigen-basis gains the phase theta_jk = dt E (lam_j - lam_k)/hbar, the
  // sum of consecutive angles E kappa_q.  Each phase is kept as
  // (cos - 1, sin) from a half-angle sincos so that the rotation is applied
  // as a small increment.
  static __device__ __forceinline__ void rotate(R (&y)[MA], R e, const R *__restrict__ mt) {
    if constexpr (N >= 2) {
      R cm[N - 1], sn[N - 1];
#pragma unroll
      for (int q = 0; q < N - 1; ++q) {
        R half = e * mt[kCoefKap + q] * R(0.5);
        R s, c;
        sincos_r(half, &s, &c);
        sn[q] = R(2) * s * c;
        cm[q] = R(-2) * s * s;
      }
#pragma unroll
      for (int j = 0; j < N - 1; ++j) {
        R pc = cm[j], ps = sn[j];
#pragma unroll
        for (int k = j + 1; k < N; ++k) {
          if (k > j + 1) {
            // (1 + pc + i ps)(1 + cm + i sn) = 1 + (pc + cm + pc cm - ps sn) + i (ps + sn + ps cm + pc sn)
            R c2 = cm[k - 1], s2 = sn[k - 1];
            R nc = fma(pc, c2, fma(-ps, s2, pc + c2));
            R ns = fma(ps, c2, fma(pc, s2, ps + s2));
            pc = nc;
            ps = ns;
          }
          const int p = k * (k - 1) / 2 + j;
          const int ir = N - 1 + 2 * p, ii = ir + 1;
          R re = y[ir], im = y[ii];
          y[ir] = re + fma(re, pc, -(im * ps));
          y[ii] = im + fma(re, ps, im * pc);
        }
      }
    }
  }

  // polarization current n3D tr{mu L0(rho^{n+1/2})} = at . y + p0
  static __device__ __forceinline__ R polar(const R (&y)[MA], const R *__restrict__ mt) {
    R acc = mt[coef_p0(N)];
#pragma unroll
    for (int j = 0; j < M; ++j) acc = fma(mt[coef_at(N) + j], y[j], acc);
    return acc;
  }

  // sigma_{n+1} = e^{L0 dt} y = y + (bf + am y)
  static __device__ __forceinline__ void propagate(R (&y)[MA], const R *__restrict__ mt) {
    R out[MA];
#pragma unroll
    for (int i = 0; i < M; ++i) {
      R acc = mt[coef_bf(N) + i];
#pragma unroll
      for (int j = 0; j < M; ++j) acc = fma(mt[coef_am(N) + i * M + j], y[j], acc);
      out[i] = y[i] + acc;
    }
#pragma unroll
    for (int i = 0; i < M; ++i) y[i] = out[i];
  }

  static __device__ __forceinline__ double readout(const R (&y)[MA], const double *__restrict__ ro) {
    double acc = ro[0];
#pragma unroll
    for (int j = 0; j < M; ++j) acc = fma(ro[1 + j], double(y[j]), acc);
    return acc;
  }
};

__device__ __forceinline__ bool due(int64_t n1, int64_t interval) { return n1 % interval == 0; }

// density records of one cell at local step n (values of rho^{n+1/2})
template <int N, typename R>
__device__ __forceinline__ void record_density(const DevSim &sim, int64_t c, int64_t n1, int mat,
                                               const R (&y)[Cell<N, R>::MA]) {
  constexpr int M = Cell<N, R>::M;
  if (sim.rec_first) {
    const int32_t b = sim.rec_first[c], e = sim.rec_first[c + 1];
    for (int32_t r = b; r < e; ++r) {
      const DevRecord &rc = sim.rec[sim.rec_ids[r]];
      if (rc.quantity < 2 || !due(n1, rc.interval)) continue;
      rc.out[n1 / rc.interval - 1] = Cell<N, R>::readout(y, rc.readout + int64_t(mat) * (M + 1));
    }
  }
  for (int32_t r = 0; r < sim.n_rec_all; ++r) {
    const DevRecord &rc = sim.rec[sim.rec_all[r]];
    if (rc.quantity < 2 || !due(n1, rc.interval)) continue;
    rc.out[(n1 / rc.interval - 1) * sim.nx + c] = Cell<N, R>::readout(y, rc.readout + int64_t(mat) * (M + 1));
  }
}

// field records (E^{n+1}, H^{n+1/2}) and zero density values outside quantum cells
template <typename R>
__device__ __forceinline__ void record_fields(const DevSim &sim, int64_t c, int64_t n1, R e, R h,
                                              bool qm) {
  auto val = [&](const DevRecord &rc, double &v) -> bool {
    if (rc.quantity == 0) { v = double(e); return true; }
    if (rc.quantity == 1) { v = double(h); return true; }
    if (!qm) { v = 0.0; return true; }
    return false;
  };
  if (sim.rec_first) {
    const int32_t b = sim.rec_first[c], en = sim.rec_first[c + 1];
    for (int32_t r = b; r < en; ++r) {
      const DevRecord &rc = sim.rec[sim.rec_ids[r]];
      double v;
      if (!due(n1, rc.interval) || !val(rc, v)) continue;
      rc.out[n1 / rc.interval - 1] = v;
    }
  }
  for (int32_t r = 0; r < sim.n_rec_all; ++r) {
    const DevRecord &rc = sim.rec[sim.rec_all[r]];
    double v;
    if (!due(n1, rc.interval) || !val(rc, v)) continue;
    rc.out[(n1 / rc.interval - 1) * sim.nx + c] = v;
  }
}

template <typename R>
__device__ __forceinline__ R apply_sources(const DevSim &sim, int64_t c, int64_t n1, R e) {
  for (int32_t j = 0; j < sim.n_src; ++j) {
    const DevSource &s = sim.src[j];
    if (s.cell != c) continue;
    const R v = R(s.table[n1]);
    e = s.hard ? v : e + v;
  }
  return e;
}

// ---------------------------------------------------------------------------
// Temporally blocked kernel: one workgroup owns T = B - 2*halo consecutive
// cells of one simulation, loads them with `halo` extra cells on both sides,
// advances up to k <= halo steps with neighbour values exchanged through LDS
// (the valid region shrinks by one cell per side and step), and writes the
// owned cells to the other state buffer.
// ---------------------------------------------------------------------------
template <int N, typename R, int B>
__global__ void __launch_bounds__(B) k_blocked(const DevSim *__restrict__ sims,
                                               const DevTile *__restrict__ tiles,
                                               int64_t n0, int parity, int halo, int k) {
  using CL = Cell<N, R>;
  constexpr int M = CL::M, MA = CL::MA, S = mat_stride(N);
  __shared__ R se[B], sh[B], se2[B];
  const DevTile tile = tiles[blockIdx.x];
  const DevSim &sim = sims[tile.sim];
  const int64_t ls0 = n0 - sim.start;
  if (ls0 < 0 || ls0 >= sim.n_steps) return;
  const int ks = int(min(int64_t(k), sim.n_steps - ls0));
  const int par = parity ^ sim.parity_off;
  const int64_t nx = sim.nx;
  const R *__restrict__ e_in = static_cast<const R *>(sim.e[par]);
  const R *__restrict__ h_in = static_cast<const R *>(sim.h[par]);
  const R *__restrict__ x_in = static_cast<const R *>(sim.x[par]);
  const R *__restrict__ mtab = static_cast<const R *>(sim.mtab);
  const int l = threadIdx.x;
  const int64_t lo = int64_t(tile.c0) - halo;
  const int64_t c = lo + l;
  const bool in = c >= 0 && c < nx;
  const bool own = in && l >= halo && l < B - halo;
  int me = 0;
  R e = 0, h = 0, ca = 1, cbg = 0, cbd = 0, ch = 0;
  R x[MA];
#pragma unroll
  for (int a = 0; a < MA; ++a) x[a] = 0;
  bool qm = false;
  if (in) {
    me = sim.mat_e[c];
    const int mh = sim.mat_h[c];
    e = e_in[c];
    h = h_in[c];
    ca = mtab[me * S + kCoefA];
    cbg = mtab[me * S + kCoefBG];
    cbd = mtab[me * S + kCoefBD];
    ch = mtab[mh * S + kCoefH];
    if constexpr (N > 0) {
      qm = mtab[me * S + kCoefQM] != R(0);
      if (qm) {
#pragma unroll
        for (int a = 0; a < M; ++a) x[a] = x_in[a * nx + c];
      }
    }
  }
  const bool hcell = in && c <= nx - 2;
  const bool ecell = in && c >= 1 && c <= nx - 2;
  const bool left = in && nx > 1 && c == 0, right = in && nx > 1 && c == nx - 1;
  const bool mur_tile = nx > 1 && ((sim.edge_l == 1 && lo <= 0 && 0 < lo + B) ||
                                   (sim.edge_r == 1 && lo <= nx - 1 && nx - 1 < lo + B));
  const bool rec_any = sim.n_rec > 0;
  const R kap_l = R(sim.kap_l), kap_r = R(sim.kap_r);

  for (int s = 0; s < ks; ++s) {
    const int64_t n1 = ls0 + s + 1;
    se[l] = e;
    __syncthreads();
    const R er = l + 1 < B ? se[l + 1] : R(0);
    const R el = l > 0 ? se[l - 1] : R(0);
    if (hcell) h = fma(ch, er - e, h);
    R p = 0;
    if constexpr (N > 0) {
      uint64_t todo = __ballot(qm);
      while (todo) {
        const int lead = __ffsll(static_cast<unsigned long long>(todo)) - 1;
        const int mm = __builtin_amdgcn_readlane(me, lead);
        const bool mine = qm && me == mm;
        if (mine) {
          const R *__restrict__ mt = mtab + mm * S;
          CL::rotate(x, e, mt);
          p = CL::polar(x, mt);
          if (rec_any && own) record_density<N, R>(sim, c, n1, mm, x);
          CL::propagate(x, mt);
        }
        todo &= ~__ballot(mine);
      }
    }
    sh[l] = h;
    __syncthreads();
    const R hl = l > 0 ? sh[l - 1] : R(0);
    const R eo = e;
    if (ecell) e = fma(cbd, h - hl, fma(ca, eo, -(cbg * p)));
    if (mur_tile) {
      se2[l] = e;
      __syncthreads();
      if (left && sim.edge_l == 1) e = fma(kap_l, se2[l + 1] - eo, er);
      if (right && sim.edge_r == 1) e = fma(kap_r, se2[l - 1] - eo, el);
    }
    if ((left && sim.edge_l == 0) || (right && sim.edge_r == 0)) e = 0;
    if (in) e = apply_sources(sim, c, n1, e);
    if (rec_any && own) record_fields(sim, c, n1, e, hcell ? h : R(0), qm);
  }
  if (own) {
    R *__restrict__ e_out = static_cast<R *>(sim.e[par ^ 1]);
    R *__restrict__ h_out = static_cast<R *>(sim.h[par ^ 1]);
    R *__restrict__ x_out = static_cast<R *>(sim.x[par ^ 1]);
    e_out[c] = e;
    h_out[c] = h;
    if constexpr (N > 0) {
      if (qm) {
#pragma unroll
        for (int a = 0; a < M; ++a) x_out[a * nx + c] = x[a];
      }
    }
    if (!isfinite(double(e)) || !isfinite(double(h))) *sim.status = 1;
  }
}

// ---------------------------------------------------------------------------
// Two-launch step (Alg. 1 as written): the first kernel updates H, rho and p
// for every cell, the second E, the edges, the sources and the field records.
// E is double-buffered, H, rho and p are updated in place.
// ---------------------------------------------------------------------------
constexpr int kPlainBlock = 256;

template <int N>
__global__ void __launch_bounds__(kPlainBlock) k_plain_hd(const DevSim *__restrict__ sims,
                                                          const DevTile *__restrict__ tiles,
                                                          int64_t n0, int parity) {
  using R = double;
  using CL = Cell<N, R>;
  constexpr int M = CL::M, MA = CL::MA, S = mat_stride(N);
  const DevTile tile = tiles[blockIdx.x];
  const DevSim &sim = sims[tile.sim];
  const int64_t n = n0 - sim.start;
  if (n < 0 || n >= sim.n_steps) return;
  const int64_t nx = sim.nx;
  const int64_t c = int64_t(tile.c0) + threadIdx.x;
  if (c >= nx) return;
  const int par = parity ^ sim.parity_off;
  const R *__restrict__ e_in = static_cast<const R *>(sim.e[par]);
  R *__restrict__ hh = static_cast<R *>(sim.h[0]);
  R *__restrict__ xx = static_cast<R *>(sim.x[0]);
  R *__restrict__ pp = static_cast<R *>(sim.p);
  const R *__restrict__ mtab = static_cast<const R *>(sim.mtab);
  const R e = e_in[c];
  if (c <= nx - 2) hh[c] = fma(mtab[sim.mat_h[c] * S + kCoefH], e_in[c + 1] - e, hh[c]);
  R p = 0;
  if constexpr (N > 0) {
    const int me = sim.mat_e[c];
    const bool qm = mtab[me * S + kCoefQM] != R(0);
    uint64_t todo = __ballot(qm);
    while (todo) {
      const int lead = __ffsll(static_cast<unsigned long long>(todo)) - 1;
      const int mm = __builtin_amdgcn_readlane(me, lead);
      const bool mine = qm && me == mm;
      if (mine) {
        const R *__restrict__ mt = mtab + mm * S;
        R x[MA];
#pragma unroll
        for (int a = 0; a < M; ++a) x[a] = xx[a * nx + c];
        CL::rotate(x, e, mt);
        p = CL::polar(x, mt);
        if (sim.n_rec > 0) record_density<N, R>(sim, c, n + 1, mm, x);
        CL::propagate(x, mt);
#pragma unroll
        for (int a = 0; a < M; ++a) xx[a * nx + c] = x[a];
      }
      todo &= ~__ballot(mine);
    }
  }
  pp[c] = p;
}

__device__ __forceinline__ double plain_interior(const DevSim &sim, const double *__restrict__ e_in,
                                                 const double *__restrict__ hh,
                                                 const double *__restrict__ pp,
                                                 const double *__restrict__ mtab, int stride,
                                                 int64_t c) {
  const int me = sim.mat_e[c];
  const double ca = mtab[me * stride + kCoefA], cbg = mtab[me * stride + kCoefBG],
               cbd = mtab[me * stride + kCoefBD];
  return fma(cbd, hh[c] - hh[c - 1], fma(ca, e_in[c], -(cbg * pp[c])));
}

template <int N>
__global__ void __launch_bounds__(kPlainBlock) k_plain_e(const DevSim *__restrict__ sims,
                                                         const DevTile *__restrict__ tiles,
                                                         int64_t n0, int parity) {
  using R = double;
  constexpr int S = mat_stride(N);
  const DevTile tile = tiles[blockIdx.x];
  const DevSim &sim = sims[tile.sim];
  const int64_t n = n0 - sim.start;
  if (n < 0 || n >= sim.n_steps) return;
  const int64_t nx = sim.nx;
  const int64_t c = int64_t(tile.c0) + threadIdx.x;
  if (c >= nx) return;
  const int par = parity ^ sim.parity_off;
  const R *__restrict__ e_in = static_cast<const R *>(sim.e[par]);
  R *__restrict__ e_out = static_cast<R *>(sim.e[par ^ 1]);
  const R *__restrict__ hh = static_cast<const R *>(sim.h[0]);
  const R *__restrict__ pp = static_cast<const R *>(sim.p);
  const R *__restrict__ mtab = static_cast<const R *>(sim.mtab);
  R e = e_in[c];
  if (nx > 1) {
    if (c >= 1 && c <= nx - 2) {
      e = plain_interior(sim, e_in, hh, pp, mtab, S, c);
    } else if (c == 0) {
      e = sim.edge_l == 0 ? 0.0
                          : fma(sim.kap_l, plain_interior(sim, e_in, hh, pp, mtab, S, 1) - e_in[0], e_in[1]);
    } else {
      e = sim.edge_r == 0
              ? 0.0
              : fma(sim.kap_r, plain_interior(sim, e_in, hh, pp, mtab, S, nx - 2) - e_in[nx - 1], e_in[nx - 2]);
    }
  }
  const int64_t n1 = n + 1;
  e = apply_sources(sim, c, n1, e);
  e_out[c] = e;
  if (sim.n_rec > 0) {
    bool qm = false;
    if constexpr (N > 0) qm = mtab[sim.mat_e[c] * S + kCoefQM] != 0.0;
    record_fields(sim, c, n1, e, c <= nx - 2 ? hh[c] : 0.0, qm);
  }
  if (!isfinite(e)) *sim.status = 1;
}

template <int N, typename R>
hipError_t launch_blocked_nr(int block, const DevSim *sims, const DevTile *tiles, int n_tiles,
                             int64_t n0, int parity, int halo, int k, hipStream_t st) {
  switch (block) {
    case 64: k_blocked<N, R, 64><<<n_tiles, 64, 0, st>>>(sims, tiles, n0, parity, halo, k); break;
    case 128: k_blocked<N, R, 128><<<n_tiles, 128, 0, st>>>(sims, tiles, n0, parity, halo, k); break;
    case 256: k_blocked<N, R, 256><<<n_tiles, 256, 0, st>>>(sims, tiles, n0, parity, halo, k); break;
    case 512: k_blocked<N, R, 512><<<n_tiles, 512, 0, st>>>(sims, tiles, n0, parity, halo, k); break;
    case 1024: k_blocked<N, R, 1024><<<n_tiles, 1024, 0, st>>>(sims, tiles, n0, parity, halo, k); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename R>
hipError_t launch_blocked_r(int levels, int block, const DevSim *sims, const DevTile *tiles,
                            int n_tiles, int64_t n0, int parity, int halo, int k, hipStream_t st) {
  switch (levels) {
    case 0: return launch_blocked_nr<0, R>(block, sims, tiles, n_tiles, n0, parity, halo, k, st);
    case 2: return launch_blocked_nr<2, R>(block, sims, tiles, n_tiles, n0, parity, halo, k, st);
    case 3: return launch_blocked_nr<3, R>(block, sims, tiles, n_tiles, n0, parity, halo, k, st);
    case 4: return launch_blocked_nr<4, R>(block, sims, tiles, n_tiles, n0, parity, halo, k, st);
    case 5: return launch_blocked_nr<5, R>(block, sims, tiles, n_tiles, n0, parity, halo, k, st);
    case 6: return launch_blocked_nr<6, R>(block, sims, tiles, n_tiles, n0, parity, halo, k, st);
  }
  return hipErrorInvalidValue;
}

template <int N>
hipError_t launch_plain_n(const DevSim *sims, const DevTile *tiles, int n_tiles, int64_t n0, int parity,
                          hipStream_t st) {
  k_plain_hd<N><<<n_tiles, kPlainBlock, 0, st>>>(sims, tiles, n0, parity);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  k_plain_e<N><<<n_tiles, kPlainBlock, 0, st>>>(sims, tiles, n0, parity);
  return hipGetLastError();
}

}  // namespace

bool block_supported(int block) {
  return block == 64 || block == 128 || block == 256 || block == 512 || block == 1024;
}

int plain_block() { return kPlainBlock; }

hipError_t launch_blocked(int levels, int precision, int block, const DevSim *sims,
                          const DevTile *tiles, int n_tiles, int64_t n0, int parity, int halo, int k,
                          hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  if (k < 1 || k > halo || 2 * halo >= block) return hipErrorInvalidValue;
  if (precision == 64)
    return launch_blocked_r<double>(levels, block, sims, tiles, n_tiles, n0, parity, halo, k, st);
  return launch_blocked_r<float>(levels, block, sims, tiles, n_tiles, n0, parity, halo, k, st);
}

hipError_t launch_plain(int levels, const DevSim *sims, const DevTile *tiles, int n_tiles,
                        int64_t n0, int parity, hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  switch (levels) {
    case 0: return launch_plain_n<0>(sims, tiles, n_tiles, n0, parity, st);
    case 2: return launch_plain_n<2>(sims, tiles, n_tiles, n0, parity, st);
    case 3: return launch_plain_n<3>(sims, tiles, n_tiles, n0, parity, st);
    case 4: return launch_plain_n<4>(sims, tiles, n_tiles, n0, parity, st);
    case 5: return launch_plain_n<5>(sims, tiles, n_tiles, n0, parity, st);
    case 6: return launch_plain_n<6>(sims, tiles, n_tiles, n0, parity, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace mb
