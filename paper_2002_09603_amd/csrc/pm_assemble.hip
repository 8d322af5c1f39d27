// Element kernels, static condensation, stabilization, global assembly,
// B~_p, C~_pi and the right-hand side of one backward-Euler step.
//
// Paper references: Appendix A eq. MFE_matrix (Q1 stiffness, coupling),
// eq. MHFE_matrix (RT0 mass, A_wp, A_wpi), Sec. 2.2 eq. hmfeSys / A_33H
// (condensed blocks), Sec. 3 eq. J_def and the 3D beta_M (stabilization),
// Sec. 4 eq. app_Bp (B~_p), C~_pi = A_pipi - dt A_pip B~_p^-1 A_ppi.
//
// All assembly is a row gather (one thread per output row), so results are
// bitwise reproducible; no floating-point atomics.
#include "pm_geom.h"
#include "pm_internal.h"

namespace pm {

namespace {

// ---------------------------------------------------------------------------
// Q1 element stiffness: one thread per (local node a, cell); the thread owns
// rows 3a..3a+2 of the 24x24 K_T and integrates them with 2x2x2 Gauss.
// Ke layout: Ke[(row*24 + col)*nc + cell].
// Rows 3a..3a+2 of K_T for the hexahedron with node coordinates X; false if
// det J <= 0 at a Gauss point.
__device__ inline bool q1_rows(const double X[8][3], double Ec, double nu, int a, double K[3][24]) {
  const double lam = Ec * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  const double mu = Ec / (2.0 * (1.0 + nu));
  for (int r = 0; r < 3; ++r)
    for (int q = 0; q < 24; ++q) K[r][q] = 0.0;
  for (int q = 0; q < 8; ++q) {
    double xi[3], J[3][3], Ji[3][3];
    gauss_point(q, xi);
    const double det = jacobian(X, xi, J);
    if (!(det > 0.0)) return false;
    inv3(J, det, Ji);
    double ga[3], gr[3];
    ref_grad(a, xi, gr);
    for (int d = 0; d < 3; ++d) ga[d] = gr[0] * Ji[0][d] + gr[1] * Ji[1][d] + gr[2] * Ji[2][d];
    for (int b = 0; b < 8; ++b) {
      double gb[3];
      ref_grad(b, xi, gr);
      for (int d = 0; d < 3; ++d) gb[d] = gr[0] * Ji[0][d] + gr[1] * Ji[1][d] + gr[2] * Ji[2][d];
      const double dd = ga[0] * gb[0] + ga[1] * gb[1] + ga[2] * gb[2];
      for (int r = 0; r < 3; ++r)
        for (int s = 0; s < 3; ++s) {
          double v = lam * ga[r] * gb[s] + mu * ga[s] * gb[r];
          if (r == s) v += mu * dd;
          K[r][3 * b + s] += v * det;
        }
    }
  }
  return true;
}

__global__ void __launch_bounds__(256) k_q1_stiffness(Grid G, const double* __restrict__ coords,
                                                      const double* __restrict__ E, double nu,
                                                      double* __restrict__ Ke, int* status) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 8 * G.nc) return;
  const int a = (int)(t / G.nc);
  const int64_t c = t - (int64_t)a * G.nc;
  int i, j, k;
  G.cell_ijk(c, i, j, k);
  double X[8][3];
  load_cell_coords(G, coords, i, j, k, X);
  double K[3][24];
  if (!q1_rows(X, E[c], nu, a, K)) {
    atomicOr(status, kStatusInverted);
    return;
  }
  for (int r = 0; r < 3; ++r)
    for (int q = 0; q < 24; ++q) Ke[((size_t)(3 * a + r) * 24 + q) * G.nc + c] = K[r][q];
}

// Lattice meshes: unit-modulus stiffness of cell 0 (8 threads, one per local
// node) and its coupling column, copied from the per-cell array.
__global__ void k_q1_unit(Grid G, const double* __restrict__ coords, double nu, const double* __restrict__ ae,
                          double* __restrict__ Kh, double* __restrict__ ah, int* status) {
  const int a = threadIdx.x;
  if (a >= 8) return;
  double X[8][3];
  load_cell_coords(G, coords, 0, 0, 0, X);
  double K[3][24];
  if (!q1_rows(X, 1.0, nu, a, K)) {
    atomicOr(status, kStatusInverted);
    return;
  }
  for (int r = 0; r < 3; ++r) {
    for (int q = 0; q < 24; ++q) Kh[(3 * a + r) * 24 + q] = K[r][q];
    ah[3 * a + r] = ae[(size_t)(3 * a + r) * G.nc];
  }
}

// Per cell: coupling column a_T (24), volume, RT0 mass, its inverse, g, alpha;
// the mass itself too (36 per cell) when Mfull is not null.
__global__ void __launch_bounds__(256) k_cell_data(Grid G, const double* __restrict__ coords,
                                                   const double* __restrict__ kappa, double mu_f,
                                                   double biot, double* __restrict__ ae,
                                                   double* __restrict__ vol, double* __restrict__ Minv,
                                                   double* __restrict__ gvec, double* __restrict__ alpha,
                                                   int* status, double* __restrict__ Mfull) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= G.nc) return;
  int i, j, k;
  G.cell_ijk(c, i, j, k);
  double X[8][3];
  load_cell_coords(G, coords, i, j, k, X);
  const double kinv[3] = {mu_f / kappa[3 * c + 0], mu_f / kappa[3 * c + 1], mu_f / kappa[3 * c + 2]};
  double A[24], M[6][6], V = 0.0;
  for (int q = 0; q < 24; ++q) A[q] = 0.0;
  for (int f = 0; f < 6; ++f)
    for (int h = 0; h < 6; ++h) M[f][h] = 0.0;
  for (int q = 0; q < 8; ++q) {
    double xi[3], J[3][3], Ji[3][3];
    gauss_point(q, xi);
    const double det = jacobian(X, xi, J);
    if (!(det > 0.0)) {
      atomicOr(status, kStatusInverted);
      return;
    }
    inv3(J, det, Ji);
    V += det;
    for (int a = 0; a < 8; ++a) {
      double gr[3];
      ref_grad(a, xi, gr);
      for (int d = 0; d < 3; ++d)
        A[3 * a + d] -= biot * (gr[0] * Ji[0][d] + gr[1] * Ji[1][d] + gr[2] * Ji[2][d]) * det;
    }
    // RT0 reference basis of face f = 2d+s is cf * e_d; mapped by J / det J
    double cf[6];
    for (int d = 0; d < 3; ++d) {
      cf[2 * d + 0] = -(1.0 - xi[d]) * 0.125;
      cf[2 * d + 1] = (1.0 + xi[d]) * 0.125;
    }
    double JKJ[3][3];  // (J^T mu kappa^-1 J)[d][e]
    for (int d = 0; d < 3; ++d)
      for (int e = 0; e < 3; ++e)
        JKJ[d][e] = J[0][d] * kinv[0] * J[0][e] + J[1][d] * kinv[1] * J[1][e] + J[2][d] * kinv[2] * J[2][e];
    const double rdet = 1.0 / det;
    for (int f = 0; f < 6; ++f)
      for (int h = 0; h < 6; ++h) M[f][h] += cf[f] * cf[h] * JKJ[f >> 1][h >> 1] * rdet;
  }
  if (Mfull)
    for (int r = 0; r < 6; ++r)
      for (int s = 0; s < 6; ++s) Mfull[(size_t)(r * 6 + s) * G.nc + c] = M[r][s];
  // Cholesky M = L L^T, then M^-1 = L^-T L^-1 (symmetric by construction)
  double L[6][6];
  for (int r = 0; r < 6; ++r)
    for (int s = 0; s < 6; ++s) L[r][s] = 0.0;
  for (int r = 0; r < 6; ++r) {
    double d = M[r][r];
    for (int s = 0; s < r; ++s) d -= L[r][s] * L[r][s];
    if (!(d > 0.0)) {
      atomicOr(status, kStatusBadPivot);
      return;
    }
    L[r][r] = sqrt(d);
    for (int t = r + 1; t < 6; ++t) {
      double v = M[t][r];
      for (int s = 0; s < r; ++s) v -= L[t][s] * L[r][s];
      L[t][r] = v / L[r][r];
    }
  }
  double Li[6][6];  // L^-1 (lower)
  for (int r = 0; r < 6; ++r)
    for (int s = 0; s < 6; ++s) Li[r][s] = 0.0;
  for (int s = 0; s < 6; ++s) {
    Li[s][s] = 1.0 / L[s][s];
    for (int r = s + 1; r < 6; ++r) {
      double v = 0.0;
      for (int t = s; t < r; ++t) v -= L[r][t] * Li[t][s];
      Li[r][s] = v / L[r][r];
    }
  }
  double Mi[6][6];
  for (int r = 0; r < 6; ++r)
    for (int s = 0; s <= r; ++s) {
      double v = 0.0;
      for (int t = r; t < 6; ++t) v += Li[t][r] * Li[t][s];
      Mi[r][s] = v;
      Mi[s][r] = v;
    }
  double al = 0.0;
  for (int r = 0; r < 6; ++r) {
    double gr = 0.0;
    for (int s = 0; s < 6; ++s) {
      gr += Mi[r][s];
      Minv[(size_t)(r * 6 + s) * G.nc + c] = Mi[r][s];
    }
    gvec[(size_t)r * G.nc + c] = gr;
    al += gr;
  }
  alpha[c] = al;
  vol[c] = V;
  for (int q = 0; q < 24; ++q) ae[(size_t)q * G.nc + c] = A[q];
}

// beta_M |M| per macro-element (3D beta of Sec. 3, volume-weighted mean E)
__global__ void k_stab_weights(Grid G, const double* __restrict__ E, const double* __restrict__ vol,
                               double nu, double biot, double* __restrict__ stabw) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int mx = G.nx >> 1, my = G.ny >> 1, mz = G.nz >> 1;
  if (m >= (int64_t)mx * my * mz) return;
  const int I = (int)(m % mx), J = (int)((m / mx) % my), K = (int)(m / ((int64_t)mx * my));
  double V = 0.0, EV = 0.0;
  for (int a = 0; a < 8; ++a) {
    const int64_t c = G.cell(2 * I + (a & 1), 2 * J + ((a >> 1) & 1), 2 * K + ((a >> 2) & 1));
    V += vol[c];
    EV += E[c] * vol[c];
  }
  const double Eb = EV / V;
  const double lam = Eb * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  const double G2 = Eb / (2.0 * (1.0 + nu));
  const double beta = 9.0 * biot * biot / (32.0 * (lam + 4.0 * G2));
  stabw[m] = beta * V;
}

// Dirichlet masks
__global__ void k_masks(Grid G, int kind, uint8_t* __restrict__ ufix, uint8_t* __restrict__ pifix) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < G.nn) {
    int i, j, k;
    G.node_ijk(t, i, j, k);
    for (int d = 0; d < 3; ++d) ufix[3 * t + d] = u_fixed(G, kind, i, j, k, d);
  }
  if (t < G.nf) {
    pifix[t] = pi_fixed(G, t);
  }
}

// A_uu row counts (structured 27-point block pattern)
__global__ void k_auu_count(Grid G, int* __restrict__ cnt) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= G.nn) return;
  int i, j, k;
  G.node_ijk(n, i, j, k);
  const int cx = 1 + (i > 0) + (i < G.nx), cy = 1 + (j > 0) + (j < G.ny), cz = 1 + (k > 0) + (k < G.nz);
  cnt[n] = cx * cy * cz;
}

// A_uu row gather, one thread per (node n, neighbour offset): block (n, m) =
// sum over the cells containing both nodes of K_T[a(n), b(m)], then the
// Dirichlet identity rows / zero columns.  Blocks are placed in the row in
// (dk, dj, di) order, so consecutive threads write consecutive blocks.
// Element stiffness sources: K_T[3a+r][3b+s] = scale(T) * unit(a, b, r, s, T).
//   KeCells:   per-cell matrices, scale 1;
//   KeLattice: E_T times the 576 entries of the unit-modulus matrix (read
//              through the cache; staging them in LDS per workgroup is
//              slower).
// (On box cells the 48-value form of the unit matrix would make mirror
// images exactly equal; the A_uu hierarchy's aggregation then breaks its
// ties differently and the benchmark solve takes 84 FGMRES iterations
// instead of 81, so the assembled matrix keeps the 576 computed entries.)
struct KeCells {
  const double* Ke;
  int64_t nc;
  __device__ double scale(int64_t) const { return 1.0; }
  __device__ double unit(int a, int b, int r, int s, int64_t c) const {
    return Ke[((size_t)(3 * a + r) * 24 + 3 * b + s) * nc + c];
  }
};
struct KeLattice {
  const double* Kh;
  const double* E;
  __device__ double scale(int64_t c) const { return E[c]; }
  __device__ double unit(int a, int b, int r, int s, int64_t) const { return Kh[(3 * a + r) * 24 + 3 * b + s]; }
};

// A_uu blocks, one thread per (node, neighbour slot), a workgroup per
// kFillNodes consecutive nodes (27 threads each).  The workgroup first
// stages, for each of its nodes, the scale and index of the 8 surrounding
// cells in LDS; each thread loads its row
// position and Dirichlet flags before that barrier, then sums its 3x3 block
// over the shared cells from LDS into an LDS copy of the workgroup's rows,
// which the workgroup writes out with consecutive 8-byte stores.  Small
// workgroups (one wave) keep the barriers cheap and the LDS footprint
// small.  The column indices are written only when col is given (the
// pattern does not change between assemblies).
constexpr int kFillNodes = 2, kFillThreads = 27 * kFillNodes;

template <class KS>
__global__ void __launch_bounds__(kFillThreads) k_auu_fill(Grid G, KS Ke, const uint8_t* __restrict__ ufix,
                                                           const int* __restrict__ rowptr, int* __restrict__ col,
                                                           double* __restrict__ val) {
  __shared__ double cw[kFillNodes][8];
  __shared__ int64_t cid[kFillNodes][8];
  __shared__ double stage[kFillThreads * 9];
  const int n0 = blockIdx.x * kFillNodes;  // < nn (grid = ceil(nn / kFillNodes))
  const int base = rowptr[n0];
  const int end = rowptr[min((int64_t)n0 + kFillNodes, G.nn)];
  // the 8 cells around each of the workgroup's nodes, (ox, oy, oz) order:
  // scale (E_T on lattices, 1 otherwise; 0 outside the grid) and index
  if (threadIdx.x < 8 * kFillNodes) {
    const int ln = (int)threadIdx.x >> 3, o = (int)threadIdx.x & 7;
    const int64_t n = (int64_t)n0 + ln;
    double w = 0.0;
    int64_t c = 0;
    if (n < G.nn) {
      int i, j, k;
      G.node_ijk(n, i, j, k);
      const int ci = i - 1 + (o & 1), cj = j - 1 + ((o >> 1) & 1), ck = k - 1 + (o >> 2);
      if (ci >= 0 && ci < G.nx && cj >= 0 && cj < G.ny && ck >= 0 && ck < G.nz) {
        c = G.cell(ci, cj, ck);
        w = Ke.scale(c);
      }
    }
    cw[ln][o] = w;
    cid[ln][o] = c;
  }
  const int ln = (int)threadIdx.x / 27, q = (int)threadIdx.x - 27 * ln;
  const int64_t n = (int64_t)n0 + ln;
  const int di = q % 3 - 1, dj = (q / 3) % 3 - 1, dk = q / 9 - 1;
  int i = 0, j = 0, k = 0;
  if (n < G.nn) G.node_ijk(n, i, j, k);
  const int i2 = i + di, j2 = j + dj, k2 = k + dk;
  const bool live = n < G.nn && i2 >= 0 && i2 <= G.nx && j2 >= 0 && j2 <= G.ny && k2 >= 0 && k2 <= G.nz;
  // the row position and the Dirichlet flags are loaded before the barrier
  int pos = 0;
  int64_t m = 0;
  bool fr[3] = {false, false, false}, fm[3] = {false, false, false};
  if (live) {
    const int xlo = i > 0 ? -1 : 0, ylo = j > 0 ? -1 : 0, zlo = k > 0 ? -1 : 0;
    const int nxc = (i < G.nx ? 1 : 0) - xlo + 1, nyc = (j < G.ny ? 1 : 0) - ylo + 1;
    pos = rowptr[n] + ((dk - zlo) * nyc + (dj - ylo)) * nxc + (di - xlo);
    m = G.node(i2, j2, k2);
    for (int r = 0; r < 3; ++r) {
      fr[r] = ufix[3 * n + r];
      fm[r] = ufix[3 * m + r];
    }
  }
  __syncthreads();
  double B[9];
  for (int e = 0; e < 9; ++e) B[e] = 0.0;
  // cells (i-1+ox, j-1+oy, k-1+oz) that also contain node m, in the same
  // order (x fastest) as the diagonal kernel; corner of n: 1-o, of m: d+1-o
#pragma unroll
  for (int o = 0; o < 8; ++o) {
    const int ox = o & 1, oy = (o >> 1) & 1, oz = o >> 2;
    const double w = live ? cw[ln][o] : 0.0;
    if (w == 0.0 || ox < di || ox > di + 1 || oy < dj || oy > dj + 1 || oz < dk || oz > dk + 1) continue;
    const int64_t c = cid[ln][o];
    const int a = (1 - ox) + 2 * (1 - oy) + 4 * (1 - oz);
    const int b = (di + 1 - ox) + 2 * (dj + 1 - oy) + 4 * (dk + 1 - oz);
    for (int r = 0; r < 3; ++r)
      for (int s = 0; s < 3; ++s) B[r * 3 + s] += w * Ke.unit(a, b, r, s, c);
  }
  if (live) {
    for (int r = 0; r < 3; ++r)
      for (int s = 0; s < 3; ++s) {
        double v = (fr[r] || fm[s]) ? 0.0 : B[r * 3 + s];
        if (m == n && r == s && fr[r]) v = 1.0;
        stage[(pos - base) * 9 + r * 3 + s] = v;
      }
    if (col) col[pos] = (int)m;
  }
  __syncthreads();
  const int cnt = (end - base) * 9;
  double* dst = val + (size_t)base * 9;
  for (int e = threadIdx.x; e < cnt; e += kFillThreads) dst[e] = stage[e];
}

// Diagonal entries of A_uu (what k_auu_fill stores on the diagonal, with the
// same cell order, so the same values): B~_p needs only these, which lets the
// C~_pi set-up start before the full fill.
template <class KS>
__global__ void __launch_bounds__(256) k_auu_diag(Grid G, KS Ke, const uint8_t* __restrict__ ufix,
                                                  double* __restrict__ diag) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= G.nn) return;
  int i, j, k;
  G.node_ijk(n, i, j, k);
  double d[3] = {0.0, 0.0, 0.0};
  for (int ck = max(k - 1, 0); ck <= min(k, G.nz - 1); ++ck)
    for (int cj = max(j - 1, 0); cj <= min(j, G.ny - 1); ++cj)
      for (int ci = max(i - 1, 0); ci <= min(i, G.nx - 1); ++ci) {
        const int64_t c = G.cell(ci, cj, ck);
        const int a = (i - ci) + 2 * (j - cj) + 4 * (k - ck);
        const double w = Ke.scale(c);
        for (int r = 0; r < 3; ++r) d[r] += w * Ke.unit(a, a, r, r, c);
      }
  for (int r = 0; r < 3; ++r) diag[3 * n + r] = ufix[3 * n + r] ? 1.0 : d[r];
}

// B~_p = S|T| + dt alpha_T + (A_stab)_TT + sum_{free i} (A_up)_{iT}^2 / (A_uu)_ii
__global__ void k_bp(Grid G, const double* __restrict__ ae, const double* __restrict__ vol,
                     const double* __restrict__ alpha, const double* __restrict__ stabw,
                     const double* __restrict__ diag, const uint8_t* __restrict__ ufix, double S,
                     double dt, int stabilize, double* __restrict__ bp) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= G.nc) return;
  int i, j, k;
  G.cell_ijk(c, i, j, k);
  double v = S * vol[c] + dt * alpha[c];
  if (stabilize) v += 3.0 * stabw[G.macro(i, j, k)];
  double fs = 0.0;
  for (int a = 0; a < 8; ++a) {
    const int64_t n = G.node(i + (a & 1), j + ((a >> 1) & 1), k + ((a >> 2) & 1));
    for (int d = 0; d < 3; ++d) {
      if (ufix[3 * n + d]) continue;
      const double x = ae[(size_t)(3 * a + d) * G.nc + c];
      fs += x * x / diag[3 * n + d];
    }
  }
  bp[c] = v + fs;
}

// C~_pi rows: count, then fill (sorted columns)

// Row f of the assembled C~_pi in ascending column order without sorting:
// for a face of orientation O between the cell before it (side 0, local face
// 2O+1) and the cell after it (side 1, local face 2O), the 11 candidate
// columns (side, local face) follow a fixed order, the face itself (both
// sides' diagonal terms, side 0 first) at its place.  Absent cells and the
// Dirichlet columns (a drained top face) are skipped.  emit(col, v).
template <int O, bool VALS, class Emit>
__device__ __forceinline__ void cpi_row_sorted(const Grid& G, uint32_t i, uint32_t j, uint32_t k, uint32_t f,
                                               const double* __restrict__ Minv, const double* __restrict__ gv,
                                               const double* __restrict__ bp, double dt, Emit&& emit) {
  // slot order per orientation: (side, local face); -1 marks the diagonal
  constexpr int kSide[3][11] = {{0, -1, 1, 0, 1, 0, 1, 0, 1, 0, 1},
                                {0, 0, 1, 1, 0, -1, 1, 0, 1, 0, 1},
                                {0, 0, 1, 1, 0, 0, 1, 1, 0, -1, 1}};
  constexpr int kFace[3][11] = {{0, -1, 1, 2, 2, 3, 3, 4, 4, 5, 5},
                                {0, 1, 0, 1, 2, -1, 3, 4, 4, 5, 5},
                                {0, 1, 0, 1, 2, 3, 2, 3, 4, -1, 5}};
  constexpr int L0 = 2 * O + 1, L1 = 2 * O;
  const uint32_t pos = O == 0 ? i : (O == 1 ? j : k);
  const uint32_t lim = (uint32_t)(O == 0 ? G.nx : (O == 1 ? G.ny : G.nz));
  const bool has[2] = {pos > 0, pos < lim};
  uint32_t c[2], ck[2], F[2][6];
  c[0] = c[1] = 0;
  ck[0] = ck[1] = 0;
  const uint32_t nx = (uint32_t)G.nx, ny = (uint32_t)G.ny;
  if (has[0]) {
    const uint32_t bi = i - (O == 0), bj = j - (O == 1), bk = k - (O == 2);
    c[0] = bi + nx * (bj + ny * bk);
    ck[0] = bk;
    cell_faces32(G, bi, bj, bk, F[0]);
  }
  if (has[1]) {
    c[1] = i + nx * (j + ny * k);
    ck[1] = k;
    cell_faces32(G, i, j, k, F[1]);
  }
  auto val = [&](int sd, int l, int e) -> double {
    if (!VALS) return 0.0;
    const double sc = dt / bp[c[sd]];
    const double gl = gv[(size_t)l * G.nc + c[sd]];
    return Minv[(size_t)(l * 6 + e) * G.nc + c[sd]] - sc * gl * gv[(size_t)e * G.nc + c[sd]];
  };
#pragma unroll
  for (int q = 0; q < 11; ++q) {
    const int sd = kSide[O][q], e = kFace[O][q];
    if (sd < 0) {  // the face itself
      double v = 0.0;
      if (has[0]) v = val(0, L0, L0);
      if (has[1]) v = has[0] ? v + val(1, L1, L1) : val(1, L1, L1);
      emit(f, v);
    } else if (has[sd] && !pi_fixed_local(G, (int)ck[sd], e)) {
      emit(F[sd][e], val(sd, sd == 0 ? L0 : L1, e));
    }
  }
}

template <bool VALS, class Emit>
__device__ __forceinline__ void cpi_row_entries(const Grid& G, int64_t f, const double* __restrict__ Minv,
                                                const double* __restrict__ gv, const double* __restrict__ bp,
                                                double dt, Emit&& emit) {
  if (pi_fixed(G, f)) {
    emit((uint32_t)f, 1.0);
    return;
  }
  uint32_t i, j, k;
  const int o = face_pos(G, (uint32_t)f, i, j, k);
  if (o == 0)
    cpi_row_sorted<0, VALS>(G, i, j, k, (uint32_t)f, Minv, gv, bp, dt, emit);
  else if (o == 1)
    cpi_row_sorted<1, VALS>(G, i, j, k, (uint32_t)f, Minv, gv, bp, dt, emit);
  else
    cpi_row_sorted<2, VALS>(G, i, j, k, (uint32_t)f, Minv, gv, bp, dt, emit);
}

__global__ void k_cpi_count(Grid G, int* __restrict__ cnt) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= G.nf) return;
  int n = 0;
  cpi_row_entries<false>(G, f, nullptr, nullptr, nullptr, 0.0, [&](uint32_t, double) { ++n; });
  cnt[f] = n;
}

__global__ void __launch_bounds__(256) k_cpi_fill(Grid G, const double* __restrict__ Minv,
                                                  const double* __restrict__ gv, const double* __restrict__ bp,
                                                  double dt, const int* __restrict__ rowptr, int* __restrict__ col,
                                                  double* __restrict__ val) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= G.nf) return;
  int p = rowptr[f];
  cpi_row_entries<true>(G, f, Minv, gv, bp, dt, [&](uint32_t cl, double v) {
    col[p] = (int)cl;
    val[p] = v;
    ++p;
  });
}

// right-hand side (eq. MHFE_vector, f~_n of Sec. 2.1; no fluid source)
__global__ void k_rhs_u(Grid G, const double* __restrict__ coords, double t0, double t1, double t2,
                        const uint8_t* __restrict__ ufix, double* __restrict__ bu) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= G.nn) return;
  int i, j, k;
  G.node_ijk(n, i, j, k);
  double f[3] = {0.0, 0.0, 0.0};
  if (k == G.nz) {
    // top faces around the node: cells (ci,cj,nz-1), local face nodes 4..7
    for (int cj = max(j - 1, 0); cj <= min(j, G.ny - 1); ++cj)
      for (int ci = max(i - 1, 0); ci <= min(i, G.nx - 1); ++ci) {
        double Xf[4][3];
        for (int a = 0; a < 4; ++a) {
          const int64_t m = G.node(ci + (a & 1), cj + (a >> 1), G.nz);
          for (int d = 0; d < 3; ++d) Xf[a][d] = coords[3 * m + d];
        }
        const int la = (i - ci) + 2 * (j - cj);
        const double sa0 = (la & 1) ? 1.0 : -1.0, sa1 = (la >> 1) ? 1.0 : -1.0;
        for (int q = 0; q < 4; ++q) {
          const double x = (q & 1) ? kGauss : -kGauss, y = (q >> 1) ? kGauss : -kGauss;
          double tx[3] = {0, 0, 0}, ty[3] = {0, 0, 0};
          for (int a = 0; a < 4; ++a) {
            const double s0 = (a & 1) ? 1.0 : -1.0, s1 = (a >> 1) ? 1.0 : -1.0;
            const double dx = 0.25 * s0 * (1.0 + s1 * y), dy = 0.25 * s1 * (1.0 + s0 * x);
            for (int d = 0; d < 3; ++d) {
              tx[d] += dx * Xf[a][d];
              ty[d] += dy * Xf[a][d];
            }
          }
          const double cx = tx[1] * ty[2] - tx[2] * ty[1], cy = tx[2] * ty[0] - tx[0] * ty[2],
                       cz = tx[0] * ty[1] - tx[1] * ty[0];
          const double dS = sqrt(cx * cx + cy * cy + cz * cz);
          const double N = 0.25 * (1.0 + sa0 * x) * (1.0 + sa1 * y);
          f[0] += N * t0 * dS;
          f[1] += N * t1 * dS;
          f[2] += N * t2 * dS;
        }
      }
  }
  for (int d = 0; d < 3; ++d) bu[3 * n + d] = ufix[3 * n + d] ? 0.0 : f[d];
}

__global__ void k_rhs_p(Grid G, const double* __restrict__ ae, const double* __restrict__ vol,
                        const double* __restrict__ gv, const double* __restrict__ stabw,
                        const uint8_t* __restrict__ pifix, const double* __restrict__ u_prev,
                        const double* __restrict__ p_prev, double S, double dt, double p_top,
                        int stab_rhs, double* __restrict__ bpv) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= G.nc) return;
  int i, j, k;
  G.cell_ijk(c, i, j, k);
  double v = 0.0;
  if (u_prev) {
    for (int a = 0; a < 8; ++a) {
      const int64_t n = G.node(i + (a & 1), j + ((a >> 1) & 1), k + ((a >> 2) & 1));
      for (int d = 0; d < 3; ++d) v -= ae[(size_t)(3 * a + d) * G.nc + c] * u_prev[3 * n + d];
    }
  }
  if (p_prev) {
    v += S * vol[c] * p_prev[c];
    if (stab_rhs) {
      const double w = stabw[G.macro(i, j, k)];
      const double pc = p_prev[c];
      v += w * ((pc - p_prev[G.cell(i ^ 1, j, k)]) + (pc - p_prev[G.cell(i, j ^ 1, k)]) +
                (pc - p_prev[G.cell(i, j, k ^ 1)]));
    }
  }
  // lifting of the prescribed face pressures: -dt * (-g_T) p_top on drained faces
  int64_t F[6];
  G.cell_faces(i, j, k, F);
  for (int e = 0; e < 6; ++e)
    if (pifix[F[e]]) v += dt * gv[(size_t)e * G.nc + c] * p_top;
  bpv[c] = v;
}

__global__ void k_rhs_pi(Grid G, const double* __restrict__ Minv, const uint8_t* __restrict__ pifix,
                         double p_top, double* __restrict__ bpi) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= G.nf) return;
  if (pifix[f]) {
    bpi[f] = p_top;
    return;
  }
  double v = 0.0;
  int64_t cc[2];
  int lf[2];
  G.face_cells(f, cc, lf);
  for (int s = 0; s < 2; ++s) {
    const int64_t c = cc[s];
    if (c < 0) continue;
    int i, j, k;
    G.cell_ijk(c, i, j, k);
    int64_t F[6];
    G.cell_faces(i, j, k, F);
    for (int e = 0; e < 6; ++e)
      if (pifix[F[e]]) v -= Minv[(size_t)(lf[s] * 6 + e) * G.nc + c] * p_top;
  }
  bpi[f] = v;
}

}  // namespace

// the element stiffness source of the context (see KeCells / KeLattice)
template <class F>
void with_element_source(const pm_ctx* c, F&& f) {
  if (c->lattice)
    f(KeLattice{c->lat.Kh, c->E});
  else
    f(KeCells{c->Ke, c->nc});
}

Grid grid_of(const pm_ctx* c) {
  Grid G;
  G.nx = c->nx;
  G.ny = c->ny;
  G.nz = c->nz;
  G.drained = c->bc_kind != PM_BC_CANTILEVER;
  G.nn = c->nn;
  G.nc = c->nc;
  G.nfx = c->nfx;
  G.nfy = c->nfy;
  G.nfz = c->nfz;
  G.nf = c->nf;
  G.dnx.init((uint32_t)c->nx);
  G.dnx1.init((uint32_t)c->nx + 1);
  G.dny.init((uint32_t)c->ny);
  G.dny1.init((uint32_t)c->ny + 1);
  return G;
}

int check_status(pm_ctx* c, const char* where) {
  int st = 0;
  PM_HIP(hipMemcpyAsync(&st, c->status, sizeof(int), hipMemcpyDeviceToHost, c->s));
  PM_HIP(hipStreamSynchronize(c->s));
  if (st & kStatusInverted)
    throw Error(PM_EINVAL, std::string(where) + ": non-positive Jacobian determinant (inverted hexahedron)");
  if (st & kStatusBadPivot)
    throw Error(PM_EINVAL, std::string(where) + ": RT0 mass matrix not positive definite");
  if (st & kStatusNonFinite) throw Error(PM_EBREAKDOWN, std::string(where) + ": non-finite value");
  if (st & kStatusCapacity) throw Error(PM_EINTERNAL, std::string(where) + ": internal capacity exceeded");
  return st;
}

// On an axis-aligned box with a diagonal permeability the RT0 basis
// functions of faces of different directions are orthogonal in the K^-1
// weighted product, so M_T, and M_T^-1, couple only the two faces of each
// direction.  The computed matrices carry rounding-level off-block entries
// (from the Jacobian's off-diagonal rounding).  k_minv_pattern flags a cell
// whose off-block entries exceed 1e-12 of the geometric mean of the two
// diagonals (|m_ab| <= sqrt(m_aa m_bb) for an SPD matrix; NaN flags too).
// Without a flag the operator applications use the direction blocks only;
// M^-1 itself, g, alpha and the assembled C~_pi keep every entry (the AMG
// set-up sees the same matrix either way).
__global__ void k_minv_pattern(Grid G, const double* __restrict__ Minv, int* status) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool full = false;
  if (c < G.nc) {
    double dg[6];
    for (int a = 0; a < 6; ++a) dg[a] = Minv[(size_t)(a * 7) * G.nc + c];
    for (int a = 0; a < 6; ++a)
      for (int b = a + 1; b < 6; ++b)
        if ((a >> 1) != (b >> 1)) {
          const double m = fabs(Minv[(size_t)(a * 6 + b) * G.nc + c]);
          full |= !(m <= 1e-12 * sqrt(dg[a] * dg[b]));
        }
  }
  if (__ballot(full) != 0ull && (threadIdx.x & 63) == 0) atomicOr(status, kStatusFullMinv);
}

void build_cpi(pm_ctx* c, hipStream_t s) {
  const Grid G = grid_of(c);
  k_bp<<<blocks_for(G.nc), kBlock, 0, s>>>(G, c->ae, c->vol, c->alpha, c->stabw, c->auu_diag, c->ufix,
                                           c->S, c->dt, c->opts.stabilize, c->bp);
  PM_CHECK_LAUNCH();
  if (!c->Cpi.rowptr) {
    c->Cpi.bs = 1;
    c->Cpi.n = c->Cpi.m = (int)G.nf;
    c->Cpi.rowptr = dalloc<int>(G.nf + 1);
    int* cnt = dalloc<int>(G.nf);
    k_cpi_count<<<blocks_for(G.nf), kBlock, 0, s>>>(G, cnt);
    PM_CHECK_LAUNCH();
    int total = 0;
    exclusive_scan(s, cnt, c->Cpi.rowptr, (int)G.nf, &total);
    dfree(cnt);
    c->Cpi.nnzb = total;
    c->Cpi.col = dalloc<int>(total);
    c->Cpi.val = dalloc<double>(total);
  }
  k_cpi_fill<<<blocks_for(G.nf), kBlock, 0, s>>>(G, c->Minv, c->g, c->bp, c->dt, c->Cpi.rowptr, c->Cpi.col,
                                                 c->Cpi.val);
  PM_CHECK_LAUNCH();
}

void assemble_all(pm_ctx* c) {
  const Grid G = grid_of(c);
  hipStream_t s = c->s;
  PM_HIP(hipMemsetAsync(c->status, 0, sizeof(int), s));
  k_masks<<<blocks_for(std::max(G.nn, G.nf)), kBlock, 0, s>>>(G, c->bc_kind, c->ufix, c->pifix);
  PM_CHECK_LAUNCH();
  k_cell_data<<<blocks_for(G.nc), kBlock, 0, s>>>(G, c->coords, c->kappa, c->mu, c->biot, c->ae, c->vol,
                                                  c->Minv, c->g, c->alpha, c->status, nullptr);
  PM_CHECK_LAUNCH();
  c->Mq_valid = false;
  c->mfe_valid = false;
  if (c->opts.block_minv) {
    k_minv_pattern<<<blocks_for(G.nc), kBlock, 0, s>>>(G, c->Minv, c->status);
    PM_CHECK_LAUNCH();
  }
  if (c->lattice) {
    if (!c->lat.Kh) {
      c->lat.Kh = dalloc<double>(576);
      c->lat.ah = dalloc<double>(24);
    }
    k_q1_unit<<<1, 64, 0, s>>>(G, c->coords, c->nu, c->ae, c->lat.Kh, c->lat.ah, c->status);
  } else {
    k_q1_stiffness<<<blocks_for(8 * G.nc), kBlock, 0, s>>>(G, c->coords, c->E, c->nu, c->Ke, c->status);
  }
  PM_CHECK_LAUNCH();
  const int st = check_status(c, "element kernels");
  if (c->lattice) lattice_unit(c);
  c->mblock = c->opts.block_minv && !(st & kStatusFullMinv);
  k_stab_weights<<<blocks_for(c->nmacro), kBlock, 0, s>>>(G, c->E, c->vol, c->nu, c->biot, c->stabw);
  PM_CHECK_LAUNCH();
  if (!c->Auu.rowptr) {
    c->Auu.bs = 3;
    c->Auu.n = c->Auu.m = (int)G.nn;
    c->Auu.rowptr = dalloc<int>(G.nn + 1);
    int* cnt = dalloc<int>(G.nn);
    k_auu_count<<<blocks_for(G.nn), kBlock, 0, s>>>(G, cnt);
    PM_CHECK_LAUNCH();
    int total = 0;
    exclusive_scan(s, cnt, c->Auu.rowptr, (int)G.nn, &total);
    dfree(cnt);
    c->Auu.nnzb = total;
    c->Auu.col = dalloc<int>(total);
    c->auu_cols_set = false;
    c->Auu.val = dalloc<double>((int64_t)total * 9);
  }
  with_element_source(c, [&](auto K) {
    k_auu_diag<<<blocks_for(G.nn), kBlock, 0, s>>>(G, K, c->ufix, c->auu_diag);
  });
  PM_CHECK_LAUNCH();
}

// The per-cell data again, with the RT0 mass stored in Mfull (36 per cell,
// [r*6+s][cell]); the other outputs are rewritten with the same values.
void cell_data(pm_ctx* c, double* Mfull) {
  const Grid G = grid_of(c);
  hipStream_t s = c->s;
  PM_HIP(hipMemsetAsync(c->status, 0, sizeof(int), s));
  k_cell_data<<<blocks_for(G.nc), kBlock, 0, s>>>(G, c->coords, c->kappa, c->mu, c->biot, c->ae, c->vol,
                                                  c->Minv, c->g, c->alpha, c->status, Mfull);
  PM_CHECK_LAUNCH();
  check_status(c, "element kernels");
}

// Values of A_uu, the FP32 lattice data and the packed M_T^-1 (after
// assemble_all; the A_uu hierarchy and the solve need them, C~_pi does not).
void assemble_auu(pm_ctx* c) {
  const Grid G = grid_of(c);
  hipStream_t s = c->s;
  int* col = c->auu_cols_set ? nullptr : c->Auu.col;
  with_element_source(c, [&](auto K) {
    k_auu_fill<<<(G.nn + kFillNodes - 1) / kFillNodes, kFillThreads, 0, s>>>(G, K, c->ufix, c->Auu.rowptr, col,
                                                                           c->Auu.val);
  });
  c->auu_cols_set = true;
  PM_CHECK_LAUNCH();
  if (c->lattice) lattice_finish(c);
  pack_minv(c);
}


void build_rhs(pm_ctx* c, const double* u_prev, const double* p_prev, double* b) {
  const Grid G = grid_of(c);
  hipStream_t s = c->s;
  k_rhs_u<<<blocks_for(G.nn), kBlock, 0, s>>>(G, c->coords, c->trac[0], c->trac[1], c->trac[2], c->ufix, b);
  PM_CHECK_LAUNCH();
  k_rhs_p<<<blocks_for(G.nc), kBlock, 0, s>>>(G, c->ae, c->vol, c->g, c->stabw, c->pifix, u_prev, p_prev,
                                              c->S, c->dt, c->p_top,
                                              (c->opts.stabilize && c->opts.increment_stab) ? 1 : 0,
                                              b + c->n_u);
  PM_CHECK_LAUNCH();
  k_rhs_pi<<<blocks_for(G.nf), kBlock, 0, s>>>(G, c->Minv, c->pifix, c->p_top, b + c->n_u + c->n_p);
  PM_CHECK_LAUNCH();
}

}  // namespace pm
