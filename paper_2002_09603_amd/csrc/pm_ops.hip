// Block operator A_H (eq. stab_A) and its transpose, the block upper
// triangular preconditioner M^-1 of eq. hybridPrec (back substitution
// pi -> p -> u) and M^-T (forward substitution u -> p -> pi), the cell flux
// reconstruction of Sec. 2.2 and the adjoint gradient kernels.
//
// The u-rows use the assembled A_uu (sliced ELL, fused with the coupling
// gather); the p- and pi-rows are applied element by element from the
// per-cell data (coupling column a_T, RT0 inverse mass, g_T = M_T^-1 1,
// alpha_T, beta_M |M|) with implicit structured indexing: this moves fewer
// bytes than assembled CSR for these blocks and needs no index arrays.
// Dirichlet dofs are identity rows with zeroed columns (masks ufix, pifix).
#include "pm_internal.h"

namespace pm {

namespace {

// coupling columns a_T: per-cell array, or one column for every cell of a lattice
struct AeCells {
  const double* ae;
  int64_t nc;
  __device__ double operator()(int q, int64_t c) const { return ld32(ae + (size_t)q * nc, (uint32_t)c); }
};
struct AeLattice {
  const double* ah;
  __device__ double operator()(int q, int64_t) const { return ah[q]; }
};

// u-rows: y_u = A_uu u + sgn * A_up p     (sgn = +1: A_H; -1: A_H^T, since A_pu = -A_up^T)
template <class T>
__global__ void __launch_bounds__(256) k_ah_u(Grid G, int n, const int* __restrict__ sptr,
                                              const int* __restrict__ perm, const int* __restrict__ col,
                                              const T* __restrict__ val,
                                              const double* __restrict__ ae, const uint8_t* __restrict__ ufix,
                                              const T* __restrict__ u, const T* __restrict__ p, double sgn,
                                              T* __restrict__ y) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = t / kSlice, lane = t % kSlice;
  if (s * kSlice >= n) return;
  const int e0 = sptr[s], e1 = sptr[s + 1];
  double acc[3] = {0.0, 0.0, 0.0};
  sell_row<3, 3, T, double>(e0, e1, col, val, u, lane, acc);
  const int r = sell_row_of(perm, t, n);
  if (r < 0) return;
  int i, j, k;
  G.node_ijk(r, i, j, k);
  double cp[3] = {0.0, 0.0, 0.0};
  for (int ck = max(k - 1, 0); ck <= min(k, G.nz - 1); ++ck)
    for (int cj = max(j - 1, 0); cj <= min(j, G.ny - 1); ++cj)
      for (int ci = max(i - 1, 0); ci <= min(i, G.nx - 1); ++ci) {
        const int64_t c = G.cell(ci, cj, ck);
        const int a = (i - ci) + 2 * (j - cj) + 4 * (k - ck);
        const double pc = (double)p[c];
        for (int d = 0; d < 3; ++d) cp[d] += ae[(size_t)(3 * a + d) * G.nc + c] * pc;
      }
  for (int d = 0; d < 3; ++d) {
    const size_t q = 3 * (size_t)r + d;
    y[q] = (T)(acc[d] + (ufix[q] ? 0.0 : sgn * cp[d]));
  }
}

// p-rows: y_p = su * sum a_T u + (S|T| + dt alpha) p + A_stab p + spi * sum_e (-g_e) pi_e
//   A_H:   su = -1, spi = dt      A_H^T: su = +1, spi = 1
// Dirichlet columns follow u_fixed / pi_fixed_local (the rule the masks are
// built from); all indices are 32-bit offsets from wave-uniform bases.
template <class T, class AE>
__global__ void __launch_bounds__(256) k_ah_p(Grid G, int kind, AE ae, const double* __restrict__ vol,
                                              const double* __restrict__ alpha, const double* __restrict__ gv,
                                              const double* __restrict__ stabw, const T* __restrict__ u,
                                              const T* __restrict__ p, const T* __restrict__ pi, double S,
                                              double dt, int stabilize, double su, double spi,
                                              double* __restrict__ y) {
  const int64_t c64 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c64 >= G.nc) return;
  const uint32_t c = (uint32_t)c64;
  int i, j, k;
  G.cell_ijk(c64, i, j, k);
  const uint32_t sy = (uint32_t)G.nx + 1, sz = sy * ((uint32_t)G.ny + 1);
  const uint32_t n0 = (uint32_t)i + sy * (uint32_t)j + sz * (uint32_t)k;
  double v = 0.0;
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
    const uint32_t n = n0 + (uint32_t)ax + (ay ? sy : 0u) + (az ? sz : 0u);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double t = ae(3 * a + d, c) * (double)ld32(u, 3 * n + d);
      if (!u_fixed(G, kind, i + ax, j + ay, k + az, d)) v += t;
    }
  }
  v *= su;
  const double pc = (double)ld32(p, c);
  v += (S * ld32(vol, c) + dt * ld32(alpha, c)) * pc;
  if (stabilize) {
    const uint32_t nx = (uint32_t)G.nx, nxy = nx * (uint32_t)G.ny;
    const uint32_t mx = nx >> 1, my = (uint32_t)G.ny >> 1;
    const double w = ld32(stabw, ((uint32_t)i >> 1) + mx * (((uint32_t)j >> 1) + my * ((uint32_t)k >> 1)));
    // partners in the 2x2x2 macro-element: cells (i^1,j,k), (i,j^1,k), (i,j,k^1)
    const uint32_t cx = (i & 1) ? c - 1 : c + 1, cy = (j & 1) ? c - nx : c + nx, cz = (k & 1) ? c - nxy : c + nxy;
    v += w * ((pc - (double)ld32(p, cx)) + (pc - (double)ld32(p, cy)) + (pc - (double)ld32(p, cz)));
  }
  uint32_t F[6];
  cell_faces32(G, (uint32_t)i, (uint32_t)j, (uint32_t)k, F);
  double t = 0.0;
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    const double q = ld32(gv + (size_t)e * G.nc, c) * (double)ld32(pi, F[e]);
    if (!pi_fixed_local(G, k, e)) t -= q;
  }
  y[c] = v + spi * t;
}

// pi-rows: y_pi = sp * sum_T (-g_T[lf]) p_T + sum_T M_T^-1 pi_T (free faces);  fixed: y = pi
//   A_H: sp = 1    A_H^T: sp = dt
// M_T^-1 is read from its packed upper triangle (21 values per cell).
template <class T>
struct AhPiTerm {
  const Grid& G;
  const double* __restrict__ Mp;
  const double* __restrict__ gv;
  const T* __restrict__ p;
  const T* __restrict__ pi;
  double sp;
  template <int L>
  __device__ __forceinline__ double operator()(LocalFace<L>, uint32_t c, const uint32_t F[6], uint32_t ck) const {
    double v = -sp * ld32(gv + (size_t)L * G.nc, c) * (double)ld32(p, c);
#pragma unroll
    for (int e = 0; e < 6; ++e) {
      const double t = ld32(Mp + (size_t)sym6(L < e ? L : e, L < e ? e : L) * G.nc, c) * (double)ld32(pi, F[e]);
      if (!pi_fixed_local(G, (int)ck, e)) v += t;  // a drained top face is a zero column
    }
    return v;
  }
};

// one thread per cell, writing the rows of the faces it owns
template <class T>
__global__ void __launch_bounds__(256) k_ah_pi(Grid G, const double* __restrict__ Mp,
                                               const double* __restrict__ gv, const T* __restrict__ p,
                                               const T* __restrict__ pi, double sp, double* __restrict__ y) {
  const int64_t c = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (c >= G.nc) return;
  int i, j, k;
  G.cell_ijk(c, i, j, k);
  owned_face_rows<double>(G, (uint32_t)i, (uint32_t)j, (uint32_t)k, AhPiTerm<T>{G, Mp, gv, p, pi, sp},
                          [&](uint32_t f, bool fixed, double acc) { y[f] = fixed ? (double)pi[f] : acc; });
}

// The same rows when M_T^-1 couples only the two faces of each direction
// (up to rounding-level entries, which are left out): local face L = 2d + s
// meets faces 2d and 2d+1 through the block [[m0, m1], [m1, m2]] of
// direction d (Mb[3d + q]), and g_L = M^-1 1 is the block's row sum.
template <class T>
struct AhPiBlockTerm {
  const Grid& G;
  const double* __restrict__ Mb;
  const T* __restrict__ p;
  const T* __restrict__ pi;
  double sp;
  template <int L>
  __device__ __forceinline__ double operator()(LocalFace<L>, uint32_t c, const uint32_t F[6], uint32_t ck) const {
    constexpr int d = L >> 1, sd = L & 1;
    const double md = ld32(Mb + (size_t)(3 * d + 2 * sd) * G.nc, c);
    const double mo = ld32(Mb + (size_t)(3 * d + 1) * G.nc, c);
    const double gl = sd ? mo + md : md + mo;
    double v = -sp * gl * (double)ld32(p, c);
    v += (sd ? mo : md) * (double)ld32(pi, F[2 * d]);
    // a drained top face is a zero column
    if (!pi_fixed_local(G, (int)ck, 2 * d + 1)) v += (sd ? md : mo) * (double)ld32(pi, F[2 * d + 1]);
    return v;
  }
};

template <class T>
__global__ void __launch_bounds__(256) k_ah_pi_block(Grid G, const double* __restrict__ Mb,
                                                     const T* __restrict__ p, const T* __restrict__ pi, double sp,
                                                     double* __restrict__ y) {
  const int64_t c = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (c >= G.nc) return;
  int i, j, k;
  G.cell_ijk(c, i, j, k);
  owned_face_rows<double>(G, (uint32_t)i, (uint32_t)j, (uint32_t)k, AhPiBlockTerm<T>{G, Mb, p, pi, sp},
                          [&](uint32_t f, bool fixed, double acc) { y[f] = fixed ? (double)pi[f] : acc; });
}

// the direction blocks of M_T^-1 (its only entries beyond rounding)
__global__ void k_pack_mblock(Grid G, const double* __restrict__ Minv, double* __restrict__ Mb) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= G.nc) return;
  for (int d = 0; d < 3; ++d) {
    const int a = 2 * d, b = 2 * d + 1;
    Mb[(size_t)(3 * d + 0) * G.nc + c] = Minv[(size_t)(a * 6 + a) * G.nc + c];
    Mb[(size_t)(3 * d + 1) * G.nc + c] =
        0.5 * (Minv[(size_t)(a * 6 + b) * G.nc + c] + Minv[(size_t)(b * 6 + a) * G.nc + c]);
    Mb[(size_t)(3 * d + 2) * G.nc + c] = Minv[(size_t)(b * 6 + b) * G.nc + c];
  }
}

// packed upper triangle of the symmetrised M_T^-1
__global__ void k_pack_minv(Grid G, const double* __restrict__ Minv, double* __restrict__ Mp) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= G.nc) return;
  for (int a = 0; a < 6; ++a)
    for (int b = a; b < 6; ++b)
      Mp[(size_t)sym6(a, b) * G.nc + c] =
          0.5 * (Minv[(size_t)(a * 6 + b) * G.nc + c] + Minv[(size_t)(b * 6 + a) * G.nc + c]);
}

// preconditioner pieces -------------------------------------------------------
// z_p = (r_p - dt A_ppi z_pi) / B~_p
template <class T>
__global__ void __launch_bounds__(256) k_prec_p(Grid G, const double* __restrict__ gv, const double* __restrict__ bp,
                                                const T* __restrict__ rp, const T* __restrict__ zpi, double dt,
                                                T* __restrict__ zp) {
  const int64_t c64 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c64 >= G.nc) return;
  const uint32_t c = (uint32_t)c64;
  int i, j, k;
  G.cell_ijk(c64, i, j, k);
  uint32_t F[6];
  cell_faces32(G, (uint32_t)i, (uint32_t)j, (uint32_t)k, F);
  double t = 0.0;
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    const double q = ld32(gv + (size_t)e * G.nc, c) * (double)ld32(zpi, F[e]);
    if (!pi_fixed_local(G, k, e)) t -= q;
  }
  zp[c] = (T)(((double)ld32(rp, c) - dt * t) / ld32(bp, c));
}

// t_u = r_u - A_up z_p
template <class T, class AE>
__global__ void __launch_bounds__(256) k_prec_u(Grid G, int kind, AE ae, const T* __restrict__ ru,
                                                const T* __restrict__ zp, T* __restrict__ tu) {
  const int64_t n64 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n64 >= G.nn) return;
  const uint32_t n = (uint32_t)n64;
  int i, j, k;
  G.node_ijk(n64, i, j, k);
  // the (up to 8) cells around the node, clamped into the mesh; cells
  // outside it take p = 0
  const uint32_t nx = (uint32_t)G.nx, nxy = nx * (uint32_t)G.ny;
  const bool lx = i > 0, ly = j > 0, lz = k > 0, hx = i < G.nx, hy = j < G.ny, hz = k < G.nz;
  const uint32_t c0 = (uint32_t)(i - lx) + nx * (uint32_t)(j - ly) + nxy * (uint32_t)(k - lz);
  const uint32_t cxo = (uint32_t)(lx + hx - 1), cyo = (uint32_t)(ly + hy - 1) * nx,
                 czo = (uint32_t)(lz + hz - 1) * nxy;
  double cp[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int oz = 0; oz < 2; ++oz)
#pragma unroll
    for (int oy = 0; oy < 2; ++oy)
#pragma unroll
      for (int ox = 0; ox < 2; ++ox) {
        const bool in = (oz ? hz : lz) && (oy ? hy : ly) && (ox ? hx : lx);
        const uint32_t c = c0 + (ox ? cxo : 0u) + (oy ? cyo : 0u) + (oz ? czo : 0u);
        const double pv = (double)ld32(zp, c);
        const double pc = in ? pv : 0.0;
        const int a = (1 - ox) + 2 * (1 - oy) + 4 * (1 - oz);
#pragma unroll
        for (int d = 0; d < 3; ++d) cp[d] += ae(3 * a + d, c) * pc;
      }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const uint32_t q = 3 * n + d;
    tu[q] = (T)((double)ld32(ru, q) - (u_fixed(G, kind, i, j, k, d) ? 0.0 : cp[d]));
  }
}

// transpose pieces: z_p = (r_p - A_up^T z_u) / B~_p ;  t_pi = r_pi - dt A_ppi^T z_p
template <class T, class AE>
__global__ void k_precT_p(Grid G, AE ae, const double* __restrict__ bp,
                          const uint8_t* __restrict__ ufix, const T* __restrict__ rp, const T* __restrict__ zu,
                          T* __restrict__ zp) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= G.nc) return;
  int i, j, k;
  G.cell_ijk(c, i, j, k);
  double v = 0.0;
  for (int a = 0; a < 8; ++a) {
    const int64_t n = G.node(i + (a & 1), j + ((a >> 1) & 1), k + ((a >> 2) & 1));
    for (int d = 0; d < 3; ++d) {
      const size_t q = 3 * (size_t)n + d;
      if (!ufix[q]) v += ae(3 * a + d, c) * (double)zu[q];
    }
  }
  zp[c] = (T)(((double)rp[c] - v) / bp[c]);
}

template <class T>
__global__ void k_precT_pi(Grid G, const double* __restrict__ gv, const uint8_t* __restrict__ pifix,
                           const T* __restrict__ rpi, const T* __restrict__ zp, double dt, T* __restrict__ tpi) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= G.nf) return;
  if (pifix[f]) {
    tpi[f] = rpi[f];
    return;
  }
  int64_t cc[2];
  int lf[2];
  G.face_cells(f, cc, lf);
  double v = 0.0;
  for (int s = 0; s < 2; ++s)
    if (cc[s] >= 0) v -= gv[(size_t)lf[s] * G.nc + cc[s]] * (double)zp[cc[s]];
  tpi[f] = (T)((double)rpi[f] - dt * v);
}

__global__ void k_d2f(int64_t n, const double* __restrict__ a, float* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}
__global__ void k_f2d(int64_t n, const float* __restrict__ a, double* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (double)a[i];
}

// flux reconstruction w_T = M_T^-1 (p_T 1 - pi_T)
__global__ void k_recon_w(Grid G, const double* __restrict__ Minv, const double* __restrict__ p,
                          const double* __restrict__ pi, double* __restrict__ w) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= G.nc) return;
  int i, j, k;
  G.cell_ijk(c, i, j, k);
  int64_t F[6];
  G.cell_faces(i, j, k, F);
  double d[6];
  for (int e = 0; e < 6; ++e) d[e] = p[c] - pi[F[e]];
  for (int r = 0; r < 6; ++r) {
    double v = 0.0;
    for (int e = 0; e < 6; ++e) v += Minv[(size_t)(r * 6 + e) * G.nc + c] * d[e];
    w[6 * c + r] = v;
  }
}

// per-cell gradients (see pm_grad in poromech.h)
__global__ void k_grad(Grid G, const double* __restrict__ coords, const double* __restrict__ E, double nu,
                       const double* __restrict__ vol, const double* __restrict__ Minv,
                       const double* __restrict__ gv, const double* __restrict__ alpha,
                       const double* __restrict__ stabw, const uint8_t* __restrict__ ufix,
                       const uint8_t* __restrict__ pifix, const double* __restrict__ lam,
                       const double* __restrict__ x, const double* __restrict__ p_prev, int64_t n_u,
                       int64_t n_p, double dt, int stabilize, double* __restrict__ dk, double* __restrict__ dE) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= G.nc) return;
  int i, j, k;
  G.cell_ijk(c, i, j, k);
  const double* lu = lam;
  const double* lp = lam + n_u;
  const double* lpi = lam + n_u + n_p;
  const double* u = x;
  const double* p = x + n_u;
  const double* pi = x + n_u + n_p;
  int64_t F[6];
  G.cell_faces(i, j, k, F);
  // kappa: condensed element block (linear in kappa_T)
  const double pc = p[c];
  double rp = dt * alpha[c] * pc;
  for (int e = 0; e < 6; ++e) rp -= dt * gv[(size_t)e * G.nc + c] * pi[F[e]];
  double sk = lp[c] * rp;
  for (int r = 0; r < 6; ++r) {
    if (pifix[F[r]]) continue;
    double v = -gv[(size_t)r * G.nc + c] * pc;
    for (int e = 0; e < 6; ++e) v += Minv[(size_t)(r * 6 + e) * G.nc + c] * pi[F[e]];
    sk += lpi[F[r]] * v;
  }
  dk[c] += -sk;
  // E: Q1 stiffness energy lam^T K_T u (linear in E_T), by quadrature
  double X[8][3], ul[8][3], ll[8][3];
  load_cell_coords(G, coords, i, j, k, X);
  for (int a = 0; a < 8; ++a) {
    const int64_t n = G.node(i + (a & 1), j + ((a >> 1) & 1), k + ((a >> 2) & 1));
    for (int d = 0; d < 3; ++d) {
      ul[a][d] = u[3 * n + d];
      ll[a][d] = ufix[3 * n + d] ? 0.0 : lu[3 * n + d];
    }
  }
  const double Ec = E[c];
  const double lmb = Ec * nu / ((1.0 + nu) * (1.0 - 2.0 * nu)), mu = Ec / (2.0 * (1.0 + nu));
  double se = 0.0;
  for (int q = 0; q < 8; ++q) {
    double xi[3], J[3][3], Ji[3][3];
    gauss_point(q, xi);
    const double det = jacobian(X, xi, J);
    inv3(J, det, Ji);
    double gu[3][3] = {{0}}, gl[3][3] = {{0}};  // grad u, grad lam: [comp][dir]
    for (int a = 0; a < 8; ++a) {
      double gr[3], gx[3];
      ref_grad(a, xi, gr);
      for (int d = 0; d < 3; ++d) gx[d] = gr[0] * Ji[0][d] + gr[1] * Ji[1][d] + gr[2] * Ji[2][d];
      for (int cc = 0; cc < 3; ++cc)
        for (int d = 0; d < 3; ++d) {
          gu[cc][d] += ul[a][cc] * gx[d];
          gl[cc][d] += ll[a][cc] * gx[d];
        }
    }
    double eu[3][3], el[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        eu[a][b] = 0.5 * (gu[a][b] + gu[b][a]);
        el[a][b] = 0.5 * (gl[a][b] + gl[b][a]);
      }
    const double tu = eu[0][0] + eu[1][1] + eu[2][2], tl = el[0][0] + el[1][1] + el[2][2];
    double dd = 0.0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) dd += el[a][b] * eu[a][b];
    se += (lmb * tl * tu + 2.0 * mu * dd) * det;
  }
  double ge = -se;
  // E: stabilization coefficient of the macro-element
  if (stabilize) {
    const int i0 = i & ~1, j0 = j & ~1, k0 = k & ~1;
    int64_t mc[8];
    double W = 0.0;
    for (int a = 0; a < 8; ++a) {
      mc[a] = G.cell(i0 + (a & 1), j0 + ((a >> 1) & 1), k0 + ((a >> 2) & 1));
      W += E[mc[a]] * vol[mc[a]];
    }
    double Lq = 0.0;
    for (int a = 0; a < 8; ++a)
      for (int d = 0; d < 3; ++d) {
        const int b = a ^ (1 << d);
        if ((a >> d) & 1) continue;
        const double dpa = p[mc[a]] - (p_prev ? p_prev[mc[a]] : 0.0);
        const double dpb = p[mc[b]] - (p_prev ? p_prev[mc[b]] : 0.0);
        Lq += (lp[mc[a]] - lp[mc[b]]) * (dpa - dpb);
      }
    ge += stabw[G.macro(i, j, k)] * (Ec * vol[c] / W) * Lq;
  }
  dE[c] += ge;
}

// (d b_{n+1} / d x_n)^T lam: c_u += -A_up lam_p ; c_p += (S|T| + A_stab) lam_p
__global__ void k_rhs_adj_u(Grid G, const double* __restrict__ ae, const double* __restrict__ lp,
                            double* __restrict__ cu) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= G.nn) return;
  int i, j, k;
  G.node_ijk(n, i, j, k);
  double cp[3] = {0.0, 0.0, 0.0};
  for (int ck = max(k - 1, 0); ck <= min(k, G.nz - 1); ++ck)
    for (int cj = max(j - 1, 0); cj <= min(j, G.ny - 1); ++cj)
      for (int ci = max(i - 1, 0); ci <= min(i, G.nx - 1); ++ci) {
        const int64_t c = G.cell(ci, cj, ck);
        const int a = (i - ci) + 2 * (j - cj) + 4 * (k - ck);
        for (int d = 0; d < 3; ++d) cp[d] += ae[(size_t)(3 * a + d) * G.nc + c] * lp[c];
      }
  for (int d = 0; d < 3; ++d) cu[3 * n + d] -= cp[d];
}

__global__ void k_rhs_adj_p(Grid G, const double* __restrict__ vol, const double* __restrict__ stabw,
                            const double* __restrict__ lp, double S, int stab, double* __restrict__ cp) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= G.nc) return;
  int i, j, k;
  G.cell_ijk(c, i, j, k);
  double v = S * vol[c] * lp[c];
  if (stab) {
    const double w = stabw[G.macro(i, j, k)];
    const double l0 = lp[c];
    v += w * ((l0 - lp[G.cell(i ^ 1, j, k)]) + (l0 - lp[G.cell(i, j ^ 1, k)]) + (l0 - lp[G.cell(i, j, k ^ 1)]));
  }
  cp[c] += v;
}

template <class T>
void ah_launch(pm_ctx* c, const T* x, double* y, bool transpose) {
  const Grid G = grid_of(c);
  const T* u = x;
  const T* p = x + c->n_u;
  const T* pi = x + c->n_u + c->n_p;
  double* yu = y;
  double* yp = y + c->n_u;
  double* ypi = y + c->n_u + c->n_p;
  g_prof.begin(c->s, kProfAHu);
  if (c->lat.on) {
    lattice_ah_u<T>(c->s, G, c->lat, u, p, transpose ? -1.0 : 1.0, yu);
    // algorithmic bytes: u read, y_u written, p and E read; flops: 576 stencil
    // and 24 coupling multiply-adds per node
    g_prof.end(c->s, kProfAHu, (double)c->n_u * (sizeof(T) + 8) + (double)c->nc * (sizeof(T) + 8),
               2.0 * (576 + 24) * (double)G.nn);
  } else {
    if constexpr (sizeof(T) == 8) {
      const Sell& Auu = c->Hu.L[0].As;
      const int nth = Auu.nslices * kSlice;
      k_ah_u<double><<<blocks_for(nth), kBlock, 0, c->s>>>(G, Auu.n, Auu.sptr, Auu.perm, Auu.col, Auu.val, c->ae, c->ufix, u,
                                                           p, transpose ? -1.0 : 1.0, yu);
      // algorithmic bytes: A_uu blocks and column ids, u read, y_u written, coupling
      // columns a_T, p read, Dirichlet mask
      g_prof.end(c->s, kProfAHu,
                 (double)Auu.nnzb * (9 * 8 + 4) + (double)c->n_u * (2 * 8 + 1) + (double)c->nc * (24 * 8 + 8));
    } else {
      throw Error(PM_EINTERNAL, "A_H with FP32 input needs the lattice operator");
    }
  }
  const double su = transpose ? 1.0 : -1.0, spi = transpose ? 1.0 : c->dt;
  g_prof.begin(c->s, kProfAHp);
  if (c->lat.on)
    k_ah_p<T><<<blocks_for(G.nc), kBlock, 0, c->s>>>(G, c->bc_kind, AeLattice{c->lat.ah}, c->vol, c->alpha, c->g,
                                                     c->stabw, u, p, pi, c->S, c->dt, c->opts.stabilize, su, spi,
                                                     yp);
  else
    k_ah_p<T><<<blocks_for(G.nc), kBlock, 0, c->s>>>(G, c->bc_kind, AeCells{c->ae, G.nc}, c->vol, c->alpha, c->g,
                                                     c->stabw, u, p, pi, c->S, c->dt, c->opts.stabilize, su, spi,
                                                     yp);
  // algorithmic bytes: u, p, pi read, y_p written, |T|, alpha_T, g_T (and a_T
  // off lattices) per cell, beta_M |M| per macro-element
  g_prof.end(c->s, kProfAHp,
             (double)(c->n_u + c->n_p + c->n_pi) * sizeof(T) + 8.0 * c->n_p +
                 (double)G.nc * 8 * (8 + (c->lat.on ? 0 : 24)) + 8.0 * c->nmacro);
  g_prof.begin(c->s, kProfAHpi);
  if (c->mblock)
    k_ah_pi_block<T><<<blocks_for(G.nc), kBlock, 0, c->s>>>(G, c->Mb, p, pi, transpose ? c->dt : 1.0, ypi);
  else
    k_ah_pi<T><<<blocks_for(G.nc), kBlock, 0, c->s>>>(G, c->Mp, c->g, p, pi, transpose ? c->dt : 1.0, ypi);
  // algorithmic bytes: p, pi read, y_pi written, the per-cell matrix entries
  // (9 direction-block entries, or 21 packed M_T^-1 entries and g_T)
  g_prof.end(c->s, kProfAHpi,
             (double)(c->n_p + c->n_pi) * sizeof(T) + 8.0 * c->n_pi + (double)G.nc * 8 * (c->mblock ? 9 : 27));
  PM_CHECK_LAUNCH();
}

}  // namespace

// u-rows of A_H in FP64: y_u = A_uu u + A_up p on free rows, y_u = u on
// Dirichlet rows; the MFE system's u-rows are the same block rows
void apply_ah_u(pm_ctx* c, const double* u, const double* p, double* yu) {
  const Grid G = grid_of(c);
  if (c->lat.on) {
    lattice_ah_u<double>(c->s, G, c->lat, u, p, 1.0, yu);
  } else {
    const Sell& Auu = c->Hu.L[0].As;
    const int nth = Auu.nslices * kSlice;
    k_ah_u<double><<<blocks_for(nth), kBlock, 0, c->s>>>(G, Auu.n, Auu.sptr, Auu.perm, Auu.col, Auu.val, c->ae,
                                                         c->ufix, u, p, 1.0, yu);
    PM_CHECK_LAUNCH();
  }
}


void apply_AH(pm_ctx* c, const double* x, double* y, bool transpose) { ah_launch<double>(c, x, y, transpose); }

void apply_AH32(pm_ctx* c, const float* x, double* y, bool transpose) {
  if (c->lat.on) {
    ah_launch<float>(c, x, y, transpose);
    return;
  }
  k_f2d<<<blocks_for(c->N), kBlock, 0, c->s>>>(c->N, x, c->pw64);
  PM_CHECK_LAUNCH();
  ah_launch<double>(c, c->pw64, y, transpose);
}

template <class T>
static void prec_apply_t(pm_ctx* c, const T* r, T* z, T* tmp, bool transpose) {
  const Grid G = grid_of(c);
  hipStream_t s = c->s;
  const T* ru = r;
  const T* rp = r + c->n_u;
  const T* rpi = r + c->n_u + c->n_p;
  T* zu = z;
  T* zp = z + c->n_u;
  T* zpi = z + c->n_u + c->n_p;
  auto vc = [&](pm::Hierarchy& H, const T* b, T* x) {
    if constexpr (sizeof(T) == 8)
      amg_vcycle(s, H, (const double*)b, (double*)x);
    else
      amg_vcycle32(s, H, (const float*)b, (float*)x);
  };
  if (!transpose) {
    vc(c->Hpi, rpi, zpi);
    k_prec_p<T><<<blocks_for(G.nc), kBlock, 0, s>>>(G, c->g, c->bp, rp, zpi, c->dt, zp);
    if (c->lat.on)
      k_prec_u<T><<<blocks_for(G.nn), kBlock, 0, s>>>(G, c->bc_kind, AeLattice{c->lat.ah}, ru, zp, tmp);
    else
      k_prec_u<T><<<blocks_for(G.nn), kBlock, 0, s>>>(G, c->bc_kind, AeCells{c->ae, G.nc}, ru, zp, tmp);
    PM_CHECK_LAUNCH();
    vc(c->Hu, tmp, zu);
  } else {
    vc(c->Hu, ru, zu);
    if (c->lat.on)
      k_precT_p<T><<<blocks_for(G.nc), kBlock, 0, s>>>(G, AeLattice{c->lat.ah}, c->bp, c->ufix, rp, zu, zp);
    else
      k_precT_p<T><<<blocks_for(G.nc), kBlock, 0, s>>>(G, AeCells{c->ae, G.nc}, c->bp, c->ufix, rp, zu, zp);
    k_precT_pi<T><<<blocks_for(G.nf), kBlock, 0, s>>>(G, c->g, c->pifix, rpi, zp, c->dt, tmp);
    PM_CHECK_LAUNCH();
    vc(c->Hpi, tmp, zpi);
  }
}

void apply_Minv(pm_ctx* c, const double* r, double* z, bool transpose) {
  if (!c->opts.precond_fp32) {
    prec_apply_t<double>(c, r, z, c->pw64, transpose);
    return;
  }
  const int64_t N = c->N;
  float* rf = c->pw32;
  float* zf = c->pw32 + N;
  float* tf = c->pw32 + 2 * N;
  k_d2f<<<blocks_for(N), kBlock, 0, c->s>>>(N, r, rf);
  PM_CHECK_LAUNCH();
  prec_apply_t<float>(c, rf, zf, tf, transpose);
  k_f2d<<<blocks_for(N), kBlock, 0, c->s>>>(N, zf, z);
  PM_CHECK_LAUNCH();
}

void apply_Minv32(pm_ctx* c, const float* r, float* z, bool transpose) {
  if (!c->opts.precond_fp32) throw Error(PM_EINTERNAL, "FP32 preconditioner requested without FP32 hierarchies");
  prec_apply_t<float>(c, r, z, c->pw32 + 2 * c->N, transpose);
}

void pack_minv(pm_ctx* c) {
  const Grid G = grid_of(c);
  if (c->mblock) {
    if (!c->Mb) c->Mb = dalloc<double>(9 * G.nc);
    k_pack_mblock<<<blocks_for(G.nc), kBlock, 0, c->s>>>(G, c->Minv, c->Mb);
    PM_CHECK_LAUNCH();
    return;
  }
  if (!c->Mp) c->Mp = dalloc<double>(21 * G.nc);
  k_pack_minv<<<blocks_for(G.nc), kBlock, 0, c->s>>>(G, c->Minv, c->Mp);
  PM_CHECK_LAUNCH();
}

void reconstruct_w(pm_ctx* c, const double* p, const double* pi, double* w) {
  const Grid G = grid_of(c);
  k_recon_w<<<blocks_for(G.nc), kBlock, 0, c->s>>>(G, c->Minv, p, pi, w);
  PM_CHECK_LAUNCH();
}

void grad(pm_ctx* c, const double* lam, const double* x, const double* p_prev, double* dk, double* dE) {
  const Grid G = grid_of(c);
  k_grad<<<blocks_for(G.nc), kBlock, 0, c->s>>>(G, c->coords, c->E, c->nu, c->vol, c->Minv, c->g, c->alpha,
                                                c->stabw, c->ufix, c->pifix, lam, x,
                                                c->opts.increment_stab ? p_prev : nullptr, c->n_u, c->n_p, c->dt,
                                                c->opts.stabilize, dk, dE);
  PM_CHECK_LAUNCH();
}

void rhs_adjoint(pm_ctx* c, const double* lam, double* cvec) {
  const Grid G = grid_of(c);
  const double* lp = lam + c->n_u;
  k_rhs_adj_u<<<blocks_for(G.nn), kBlock, 0, c->s>>>(G, c->ae, lp, cvec);
  k_rhs_adj_p<<<blocks_for(G.nc), kBlock, 0, c->s>>>(G, c->vol, c->stabw, lp, c->S,
                                                     (c->opts.stabilize && c->opts.increment_stab) ? 1 : 0,
                                                     cvec + c->n_u);
  PM_CHECK_LAUNCH();
}

}  // namespace pm
