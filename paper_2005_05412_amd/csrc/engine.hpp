// Device-visible tables shared by the kernels and the host runtime.
#pragma once

#include <cstdint>

namespace mb {

// Per-material coefficient block, element type R (float or double), stride
// mat_stride(N).  The density state x (M = N*N - 1 reals) is kept in the basis
// the operators are given in; the field part is applied through the (Re, Im)
// coordinates z (K = N*(N-1) reals) of the coherences in the dipole eigenbasis.
//   [0] a'  [1] b' Gamma  [2] b'/dx  [3] c' (for H nodes)  [4] 1 if quantum
//   kappa[N-1]          dt (lam_q - lam_{q+1}) / hbar, consecutive eigenvalue gaps
//   p0, at[M], as[K]    polarization p = p0 + at . x + as . d
//   bf[M]               affine part of e^{L0 dt}
//   prop[M][M+K]        row i: (e^{L0 dt} - I)_i (M), then (e^{L0 dt} S)_i (K)
//   t0[K], tm[K][M]     z = t0 + tm x
//   sigma[N]            dt lam_j / hbar (Cayley field step)
// where d = (e^{i theta} - 1) z pairwise and S maps d back to the state
// coordinates; one step is x <- x + bf + (A - I) x + (A S) d.
constexpr int kCoefA = 0, kCoefBG = 1, kCoefBD = 2, kCoefH = 3, kCoefQM = 4, kCoefKap = 5;
__host__ __device__ constexpr int mat_m(int n) { return n > 0 ? n * n - 1 : 0; }
__host__ __device__ constexpr int mat_k(int n) { return n > 0 ? n * (n - 1) : 0; }
__host__ __device__ constexpr int coef_p0(int n) { return kCoefKap + (n > 0 ? n - 1 : 0); }
__host__ __device__ constexpr int coef_at(int n) { return coef_p0(n) + 1; }
__host__ __device__ constexpr int coef_as(int n) { return coef_at(n) + mat_m(n); }
__host__ __device__ constexpr int coef_bf(int n) { return coef_as(n) + mat_k(n); }
__host__ __device__ constexpr int coef_am(int n) { return coef_bf(n) + mat_m(n); }
__host__ __device__ constexpr int prop_w(int n) { return mat_m(n) + mat_k(n); }
__host__ __device__ constexpr int coef_t0(int n) { return coef_am(n) + mat_m(n) * prop_w(n); }
__host__ __device__ constexpr int coef_tm(int n) { return coef_t0(n) + mat_k(n); }
__host__ __device__ constexpr int coef_sg(int n) { return coef_tm(n) + mat_k(n) * mat_m(n); }
__host__ __device__ constexpr int mat_stride(int n) { return n > 0 ? coef_sg(n) + n : kCoefKap; }
// Block form of the same tables, for materials whose dipole operator is real
// and whose free propagator e^{L0 dt} couples populations only among
// themselves and each coherence only with itself (H0 diagonal, relaxation in
// rate form): then z's real parts depend only on the populations and the real
// parts of the coherences, its imaginary parts only on the imaginary parts,
// the increment maps back the same way, and A - I is one population block and
// a 2 x 2 block per pair.  P = N(N-1)/2 pairs, NP = N-1 stored populations:
//   kappa[N-1], p0, at[M], as[K]   as above (same offsets)
//   bfp[NP], ap[NP][NP]            populations: x <- y + bfp + ap y
//   blk[P][4]                      pair r: (re, im) <- y + [[b0 b1] [b2 b3]] y
//   t0r[P], tp[P][NP], tr[P][P], ti[P][P]    zr = t0r + tp x_pop + tr x_re, zi = ti x_im
//   sp[NP][P], sr[P][P], si[P][P]  y_pop = x_pop + sp dr, y_re = x_re + sr dr, y_im = x_im + si di
//   sigma[N]
__host__ __device__ constexpr int pairs_of(int n) { return n > 0 ? n * (n - 1) / 2 : 0; }
__host__ __device__ constexpr int bk_bf(int n) { return coef_as(n) + mat_k(n); }
__host__ __device__ constexpr int bk_ap(int n) { return bk_bf(n) + (n > 0 ? n - 1 : 0); }
__host__ __device__ constexpr int bk_blk(int n) { return bk_ap(n) + (n > 0 ? (n - 1) * (n - 1) : 0); }
__host__ __device__ constexpr int bk_t0(int n) { return bk_blk(n) + 4 * pairs_of(n); }
__host__ __device__ constexpr int bk_tp(int n) { return bk_t0(n) + pairs_of(n); }
__host__ __device__ constexpr int bk_tr(int n) { return bk_tp(n) + pairs_of(n) * (n > 0 ? n - 1 : 0); }
__host__ __device__ constexpr int bk_ti(int n) { return bk_tr(n) + pairs_of(n) * pairs_of(n); }
__host__ __device__ constexpr int bk_sp(int n) { return bk_ti(n) + pairs_of(n) * pairs_of(n); }
__host__ __device__ constexpr int bk_sr(int n) { return bk_sp(n) + (n > 0 ? n - 1 : 0) * pairs_of(n); }
__host__ __device__ constexpr int bk_si(int n) { return bk_sr(n) + pairs_of(n) * pairs_of(n); }
__host__ __device__ constexpr int bk_sg(int n) { return bk_si(n) + pairs_of(n) * pairs_of(n); }
__host__ __device__ constexpr int bk_stride(int n) { return n > 0 ? bk_sg(n) + n : kCoefKap; }
// coefficient stride and Cayley offset of a form
__host__ __device__ constexpr int stride_of(int n, bool bk) { return bk ? bk_stride(n) : mat_stride(n); }
__host__ __device__ constexpr int sigma_of(int n, bool bk) { return bk ? bk_sg(n) : coef_sg(n); }

// FP64 readout row of a density record (and the strong-coupling trace) per
// material: value = r0 + r . x + rs . d, length ro_len(N)
__host__ __device__ constexpr int ro_len(int n) { return mat_m(n) + 1 + mat_k(n); }
// planes of one density state buffer: FP32 keeps a compensation plane per entry
__host__ __device__ constexpr int state_planes(int n, int precision) { return (precision == 32 ? 2 : 1) * mat_m(n); }

struct DevSource {
  int64_t cell;
  int32_t hard;
  int32_t pad;
  const double *table;  // s(n dt), n = 0..n_steps
};

struct DevRecord {
  int32_t quantity;
  int32_t whole;        // 1: one value per cell per sample
  int64_t cell;
  int64_t interval;
  double *out;          // samples (x nx when whole)
  const double *readout;  // density quantities: per material ro_len(N) doubles
};

struct DevSim {
  int64_t nx, n_steps;
  int64_t start;        // engine step at which this simulation's step 0 runs
  int32_t parity_off;   // buffer parity of the engine when the simulation joined
  int32_t n_src;
  int32_t edge_l, edge_r;  // 0: perfect conductor, 1: first-order Mur, 2: impedance load
  double kap_l, kap_r;      // Mur coefficients
  double load_g_l, load_d_l, load_g_r, load_d_r;  // load edges: E' = g E + d H'_{1/2} (left), g E - d H'_{nx-3/2} (right)
  // the kernels advance E and eta0 H (eta0 = sqrt(mu0/eps0)): the update
  // coefficients are then c0 dt/(eps_r dx) and c0 dt/(mu_r dx), which FP32
  // holds exactly for the usual Courant numbers; H = h_scale x (stored value)
  double h_scale;
  // state buffers of element type R; x: M planes of nx (FP32: then M more
  // planes, the compensation of each state entry, see Cell::propagate)
  void *e[2], *h[2], *x[2];
  void *p;                   // polarization scratch of the two-launch path
  const uint8_t *mat_e, *mat_h;
  const void *mtab;
  const DevSource *src;
  const DevRecord *rec;
  int32_t n_rec, n_rec_all;
  const int32_t *rec_first;  // nx+1 offsets into rec_cell (records at one cell), or null
  const DevRecord *rec_cell; // copies of the single-cell records, grouped by cell
  const int32_t *rec_all;    // whole-domain record ids
  int32_t *status;           // kStatus* bits
  int32_t rec_every;         // gcd of the record intervals (1 when there are no records)
  int32_t cayley;            // field part by the Cayley approximant (MB_FIELD_CAYLEY)
  // strong coupling: (n3D/dt) tr{mu rho^n} per cell (FP64 ping-pong like x), each
  // buffer followed two planes on by the cell's last polarization current (the
  // start of the next step's field iteration), and per material the readout
  // (qc, aq[M], aqs[K]) from the state and the field increments
  double *qs[2];
  const double *qtab;
};

struct DevTile {
  int32_t sim;          // index in the group's simulation table
  int32_t c0;           // first output cell
  int32_t left, right;  // tiles owning the cells next to this tile's (same simulation), or -1
};

// Several chunks in one launch (a persistent launch): after each chunk a tile
// writes its owned cells, raises its flag to the chunk's epoch and waits until
// both neighbour tiles have raised theirs, so that it reloads its halo from
// finished chunks.  All tiles of the launch must be resident at once.
struct ChunkSync {
  uint32_t *flags;     // one per tile: epoch of the last chunk the tile finished (null: one chunk)
  uint32_t epoch;      // epoch of the launch's first chunk; chunk j ends at epoch + j + 1
  int32_t n_chunks;    // chunks of k steps in this launch
  int64_t spin_ticks;  // device wall-clock ticks a tile waits for a neighbour before giving up
};

// A work-queue persistent launch of a two-level and a three-level tile group
// (either may be empty): items (chunk c, tile t) in chunk-major order, handed
// out by an atomic counter; an item waits for its own tile's and both
// neighbours' items of chunk c - 1, which were handed out earlier and so are
// held by running workgroups (or done): every wait ends, whatever the grid.
struct QueueArgs {
  const DevSim *sims[2];
  const DevTile *tiles[2];
  uint32_t *flags[2];   // one per tile of each group, as in ChunkSync
  int32_t n_tiles[2];
  uint32_t *counter;    // items handed out; zero before the launch
  uint32_t epoch;       // epoch of the launch's first chunk
  int32_t n_chunks;     // chunks of k steps in this launch
  int64_t spin_ticks;
};

// bits of DevSim::status
constexpr int32_t kStatusNonFinite = 1;    // a non-finite field value was seen
constexpr int32_t kStatusWaitTimeout = 2;  // a tile gave up waiting for a neighbour tile

}  // namespace mb
