// Operator of the non-hybridized mixed system (MFE, Sec. 2.1 eq. mfeSys with
// the stabilized pressure block of Sec. 3), order [u; q; p]:
//   y_u = A_uu u + A_up p
//   y_q = A_qq q + A_qp p
//   y_p = A_pu u + dt A_pq q + (A_pp + A_stab) p
// q holds one flux per face, oriented by the face's global +x/+y/+z normal.
// On cell T the face basis is s_L times the outward RT0 basis of local face L,
// s_L = -1 on the -x, -y, -z faces and +1 on the +x, +y, +z faces, so
// A_qq = sum_T S_T M_T S_T, [A_qp]_{e,T} = -s_L and A_pq = -A_qp^T
// (Appendix A, eq. MFE_matrix, with the flux-normalised RT0 basis).
// Fixed displacements and no-flow faces are identity rows and zero columns.
#include <algorithm>
#include <utility>

#include "pm_internal.h"

namespace pm {
namespace {

__device__ __forceinline__ double face_sign(int L) { return (L & 1) ? 1.0 : -1.0; }

// a face without a drained pressure on the domain boundary carries q = 0
__device__ __forceinline__ bool q_fixed(const Grid& G, int64_t f) {
  int64_t cc[2];
  int lf[2];
  G.face_cells(f, cc, lf);
  return (cc[0] < 0 || cc[1] < 0) && !pi_fixed(G, f);
}

// face rows: y_e = sum_T s_L (sum_h s_h M_T[L][h] q_{F_T[h]} - p_T);  fixed: y_e = q_e
__global__ void __launch_bounds__(256) k_mfe_q(Grid G, const double* __restrict__ Mq, const double* __restrict__ q,
                                               const double* __restrict__ p, double* __restrict__ yq) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= G.nf) return;
  if (q_fixed(G, f)) {
    yq[f] = q[f];
    return;
  }
  int64_t cc[2];
  int lf[2];
  G.face_cells(f, cc, lf);
  double v = 0.0;
  for (int t = 0; t < 2; ++t) {
    const int64_t c = cc[t];
    if (c < 0) continue;
    const int L = lf[t];
    int i, j, k;
    G.cell_ijk(c, i, j, k);
    int64_t F[6];
    G.cell_faces(i, j, k, F);
    double r = -p[c];
    for (int h = 0; h < 6; ++h)
      if (!q_fixed(G, F[h])) r += face_sign(h) * Mq[(size_t)(L * 6 + h) * G.nc + c] * q[F[h]];
    v += face_sign(L) * r;
  }
  yq[f] = v;
}

// cell rows: y_T = -sum a_T u (free u) + dt sum_L s_L q_{F_L} (free q) + S|T| p_T + (A_stab p)_T
__global__ void __launch_bounds__(256) k_mfe_p(Grid G, int kind, const double* __restrict__ ae,
                                               const double* __restrict__ vol, const double* __restrict__ stabw,
                                               const double* __restrict__ u, const double* __restrict__ q,
                                               const double* __restrict__ p, double S, double dt, int stabilize,
                                               double* __restrict__ yp) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= G.nc) return;
  int i, j, k;
  G.cell_ijk(c, i, j, k);
  double v = 0.0;
  for (int a = 0; a < 8; ++a) {
    const int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
    const int64_t n = G.node(i + ax, j + ay, k + az);
    for (int d = 0; d < 3; ++d)
      if (!u_fixed(G, kind, i + ax, j + ay, k + az, d)) v -= ae[(size_t)(3 * a + d) * G.nc + c] * u[3 * n + d];
  }
  int64_t F[6];
  G.cell_faces(i, j, k, F);
  double div = 0.0;
  for (int L = 0; L < 6; ++L)
    if (!q_fixed(G, F[L])) div += face_sign(L) * q[F[L]];
  v += dt * div + S * vol[c] * p[c];
  if (stabilize) {
    // partners in the 2x2x2 macro-element: cells (i^1,j,k), (i,j^1,k), (i,j,k^1)
    const int64_t m = (i >> 1) + (int64_t)(G.nx >> 1) * ((j >> 1) + (int64_t)(G.ny >> 1) * (k >> 1));
    const double w = stabw[m], pc = p[c];
    v += w * ((pc - p[G.cell(i ^ 1, j, k)]) + (pc - p[G.cell(i, j ^ 1, k)]) + (pc - p[G.cell(i, j, k ^ 1)]));
  }
  yp[c] = v;
}

// L_e = sum over the face's cells T and free faces h of T of |M_T[L][h]|:
// the absolute row sum of the masked A_qq (1 on fixed faces)
__global__ void __launch_bounds__(256) k_cp_lump(Grid G, const double* __restrict__ Mq, double* __restrict__ Lq) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= G.nf) return;
  if (q_fixed(G, f)) {
    Lq[f] = 1.0;
    return;
  }
  int64_t cc[2];
  int lf[2];
  G.face_cells(f, cc, lf);
  double v = 0.0;
  for (int t = 0; t < 2; ++t) {
    const int64_t c = cc[t];
    if (c < 0) continue;
    int i, j, k;
    G.cell_ijk(c, i, j, k);
    int64_t F[6];
    G.cell_faces(i, j, k, F);
    for (int h = 0; h < 6; ++h)
      if (!q_fixed(G, F[h])) v += fabs(Mq[(size_t)(lf[t] * 6 + h) * G.nc + c]);
  }
  Lq[f] = v;
}

// neighbour of cell (i,j,k) across local face L (-1 outside the grid)
__device__ __forceinline__ int64_t cell_across(const Grid& G, int i, int j, int k, int L) {
  const int d = L >> 1, o = (L & 1) ? 1 : -1;
  const int ii = i + (d == 0 ? o : 0), jj = j + (d == 1 ? o : 0), kk = k + (d == 2 ? o : 0);
  if (ii < 0 || jj < 0 || kk < 0 || ii >= G.nx || jj >= G.ny || kk >= G.nz) return -1;
  return G.cell(ii, jj, kk);
}

__global__ void k_cp_count(Grid G, int* __restrict__ cnt) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= G.nc) return;
  int i, j, k;
  G.cell_ijk(c, i, j, k);
  int n = 1;
  for (int L = 0; L < 6; ++L) n += cell_across(G, i, j, k, L) >= 0;
  cnt[c] = n;
}

// C~_p rows in ascending column order (-z, -y, -x, self, +x, +y, +z):
//   off-diagonal across interior face e: -dt / L_e, minus the stabilization
//   weight when the neighbour is the cell's partner in its macro-element;
//   diagonal: B~_p - dt alpha (= S|T| + diag A_stab + fixed-stress term)
//   + dt sum over free faces of 1 / L_e
__global__ void __launch_bounds__(256) k_cp_fill(Grid G, const double* __restrict__ Lq,
                                                 const double* __restrict__ bp, const double* __restrict__ alpha,
                                                 const double* __restrict__ stabw, double dt, int stabilize,
                                                 const int* __restrict__ rowptr, int* __restrict__ col,
                                                 double* __restrict__ val) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= G.nc) return;
  int i, j, k;
  G.cell_ijk(c, i, j, k);
  int64_t F[6];
  G.cell_faces(i, j, k, F);
  const double w = stabilize ? stabw[(i >> 1) + (int64_t)(G.nx >> 1) * ((j >> 1) + (int64_t)(G.ny >> 1) * (k >> 1))]
                             : 0.0;
  const int ijk[3] = {i, j, k};
  double diag = bp[c] - dt * alpha[c];
  for (int L = 0; L < 6; ++L)
    if (!q_fixed(G, F[L])) diag += dt / Lq[F[L]];
  int pos = rowptr[c];
  const int order[7] = {4, 2, 0, -1, 1, 3, 5};
  for (int o = 0; o < 7; ++o) {
    const int L = order[o];
    if (L < 0) {
      col[pos] = (int)c;
      val[pos++] = diag;
      continue;
    }
    const int64_t n = cell_across(G, i, j, k, L);
    if (n < 0) continue;
    // the partner across axis d differs in bit 0 of that index: -side when odd, +side when even
    const bool partner = ((ijk[L >> 1] & 1) == 1) == ((L & 1) == 0);
    col[pos] = (int)n;
    val[pos++] = -dt / Lq[F[L]] - (partner ? w : 0.0);
  }
}

// inverse diagonal of the masked A_qq (1 on no-flow faces) and, per face,
// the Gershgorin ratio sum_j |a_ej| / a_ee of D^-1 A_qq
__global__ void __launch_bounds__(256) k_qq_diag(Grid G, const double* __restrict__ Mq, const double* __restrict__ Lq,
                                                 double* __restrict__ dinv, double* __restrict__ ratio) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= G.nf) return;
  if (q_fixed(G, f)) {
    dinv[f] = 1.0;
    ratio[f] = 1.0;
    return;
  }
  int64_t cc[2];
  int lf[2];
  G.face_cells(f, cc, lf);
  double dg = 0.0;
  for (int t = 0; t < 2; ++t)
    if (cc[t] >= 0) dg += Mq[(size_t)(lf[t] * 6 + lf[t]) * G.nc + cc[t]];
  dinv[f] = 1.0 / dg;
  ratio[f] = Lq[f] / dg;
}

// y = D^-1 A_qq x on the masked A_qq (no-flow faces: identity rows)
__global__ void __launch_bounds__(256) k_qq_dinv_apply(Grid G, const double* __restrict__ Mq,
                                                       const double* __restrict__ dinv, const double* __restrict__ x,
                                                       double* __restrict__ y) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= G.nf) return;
  if (q_fixed(G, f)) {
    y[f] = x[f];
    return;
  }
  int64_t cc[2];
  int lf[2];
  G.face_cells(f, cc, lf);
  double ax = 0.0;
  for (int t = 0; t < 2; ++t) {
    const int64_t c = cc[t];
    if (c < 0) continue;
    const int L = lf[t];
    int i, j, k;
    G.cell_ijk(c, i, j, k);
    int64_t F[6];
    G.cell_faces(i, j, k, F);
    double r = 0.0;
    for (int h = 0; h < 6; ++h)
      if (!q_fixed(G, F[h])) r += face_sign(h) * Mq[(size_t)(L * 6 + h) * G.nc + c] * x[F[h]];
    ax += face_sign(L) * r;
  }
  y[f] = dinv[f] * ax;
}

// start vector of the power iteration: a fixed sign pattern with varying
// magnitude from an integer hash of the face index
__global__ void k_qq_seed(int64_t n, double* __restrict__ v) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n) return;
  uint32_t h = (uint32_t)f * 2654435761u;
  h ^= h >> 15;
  h *= 2246822519u;
  h ^= h >> 13;
  v[f] = ((double)(h & 0xffff) / 65535.0) - 0.5;
}

// part[block] = sum over the block's entries of x^2 * s^2, x scaled by s in place
__global__ void __launch_bounds__(256) k_scale_sumsq_part(int64_t n, double* __restrict__ x, double s,
                                                          double* __restrict__ part) {
  __shared__ double sh[256];
  double m = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double v = x[i] * s;
    x[i] = v;
    m += v * v;
  }
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// part[block] = max over the block's entries of x
__global__ void __launch_bounds__(256) k_max_part(int64_t n, const double* __restrict__ x, double* __restrict__ part) {
  __shared__ double sh[256];
  double m = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) m = fmax(m, x[i]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// Chebyshev step on A_qq: r = D^-1 (b - A_qq x_in); d = c1 d + c2 r;
// x_out = x_in + d.  first: x_in = 0 (no operator application).  Face rows
// formed from the one or two cells of the face; no-flow faces are identity.
__global__ void __launch_bounds__(256) k_qq_cheb(Grid G, const double* __restrict__ Mq, const double* __restrict__ dinv,
                                                 const double* __restrict__ b, const double* __restrict__ xin,
                                                 double* __restrict__ xout, double* __restrict__ d, double c1,
                                                 double c2, int first) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= G.nf) return;
  double ax = 0.0;
  if (!first) {
    if (q_fixed(G, f)) {
      ax = xin[f];
    } else {
      int64_t cc[2];
      int lf[2];
      G.face_cells(f, cc, lf);
      for (int t = 0; t < 2; ++t) {
        const int64_t c = cc[t];
        if (c < 0) continue;
        const int L = lf[t];
        int i, j, k;
        G.cell_ijk(c, i, j, k);
        int64_t F[6];
        G.cell_faces(i, j, k, F);
        double r = 0.0;
        for (int h = 0; h < 6; ++h)
          if (!q_fixed(G, F[h])) r += face_sign(h) * Mq[(size_t)(L * 6 + h) * G.nc + c] * xin[F[h]];
        ax += face_sign(L) * r;
      }
    }
  }
  const double r = dinv[f] * (b[f] - ax);
  const double dn = (first ? 0.0 : c1 * d[f]) + c2 * r;
  d[f] = dn;
  xout[f] = (first ? 0.0 : xin[f]) + dn;
}

// right-hand side of the C~_p solve in the block lower triangular
// preconditioner: t_T = r_T - (A_pu z_u)_T - dt (A_pq z_q)_T
//                     = r_T + sum_free a_T z_u - dt sum_free-faces s_L z_q
__global__ void __launch_bounds__(256) k_btp_p(Grid G, int kind, const double* __restrict__ ae,
                                               const double* __restrict__ zu, const double* __restrict__ zq,
                                               const double* __restrict__ rp, double dt, double* __restrict__ tp) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= G.nc) return;
  int i, j, k;
  G.cell_ijk(c, i, j, k);
  double v = rp[c];
  for (int a = 0; a < 8; ++a) {
    const int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
    const int64_t n = G.node(i + ax, j + ay, k + az);
    for (int dd = 0; dd < 3; ++dd)
      if (!u_fixed(G, kind, i + ax, j + ay, k + az, dd)) v += ae[(size_t)(3 * a + dd) * G.nc + c] * zu[3 * n + dd];
  }
  int64_t F[6];
  G.cell_faces(i, j, k, F);
  double div = 0.0;
  for (int L = 0; L < 6; ++L)
    if (!q_fixed(G, F[L])) div += face_sign(L) * zq[F[L]];
  tp[c] = v - dt * div;
}

// f_q of the MFE step (Appendix A, eq. MFE_vector): on a drained face of cell
// T, -(phi_e . n, pbar) = -s_L pbar; 0 on every other face (no-flow faces are
// identity rows with zero prescribed flux)
__global__ void k_rhs_q_mfe(Grid G, double p_top, double* __restrict__ bq) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= G.nf) return;
  double v = 0.0;
  if (pi_fixed(G, f)) {
    int64_t cc[2];
    int lf[2];
    G.face_cells(f, cc, lf);
    for (int t = 0; t < 2; ++t)
      if (cc[t] >= 0) v -= face_sign(lf[t]) * p_top;
  }
  bq[f] = v;
}

void ensure_mq(pm_ctx* c) {
  if (c->Mq_valid) return;
  if (!c->Mq) c->Mq = dalloc<double>(36 * c->nc);
  cell_data(c, c->Mq);
  c->Mq_valid = true;
}

}  // namespace

// C~_p of the MFE block triangular preconditioner (Sec. 5) as CSR, rebuilt
// from the current assembly on every call
void build_cp(pm_ctx* c) {
  const Grid G = grid_of(c);
  hipStream_t s = c->s;
  ensure_mq(c);
  if (!c->Cp.rowptr) {
    c->Cp.bs = 1;
    c->Cp.n = c->Cp.m = (int)G.nc;
    c->Cp.rowptr = dalloc<int>(G.nc + 1);
    int* cnt = dalloc<int>(G.nc);
    k_cp_count<<<blocks_for(G.nc), kBlock, 0, s>>>(G, cnt);
    PM_CHECK_LAUNCH();
    int total = 0;
    exclusive_scan(s, cnt, c->Cp.rowptr, (int)G.nc, &total);
    dfree(cnt);
    c->Cp.nnzb = total;
    c->Cp.col = dalloc<int>(total);
    c->Cp.val = dalloc<double>(total);
  }
  if (!c->mfe_lq) c->mfe_lq = dalloc<double>(G.nf);
  k_cp_lump<<<blocks_for(G.nf), kBlock, 0, s>>>(G, c->Mq, c->mfe_lq);
  PM_CHECK_LAUNCH();
  k_cp_fill<<<blocks_for(G.nc), kBlock, 0, s>>>(G, c->mfe_lq, c->bp, c->alpha, c->stabw, c->dt, c->opts.stabilize,
                                                c->Cp.rowptr, c->Cp.col, c->Cp.val);
  PM_CHECK_LAUNCH();
}

// The block lower triangular preconditioner of eq. prec for the MFE system:
// C~_p and its smoothed-aggregation hierarchy, the inverse diagonal of the
// masked A_qq and the estimate of lambda_max(D^-1 A_qq) that sets the interval
// of its Chebyshev-Jacobi sweeps (the paper applies A_qq^-1 by incomplete
// Cholesky, whose triangular solves are sequential; A_qq is spectrally
// equivalent to its diagonal, so a fixed polynomial in D^-1 A_qq does the
// same job in parallel).
void mfe_prec_setup(pm_ctx* c, const AmgParams& prm) {
  const Grid G = grid_of(c);
  hipStream_t s = c->s;
  build_cp(c);
  amg_setup(s, c->Cp, prm, c->Hcp);
  constexpr int kParts = 256;
  if (!c->mfe_dqinv) c->mfe_dqinv = dalloc<double>(G.nf);
  if (!c->mfe_work) c->mfe_work = dalloc<double>(3 * G.nf + G.nc + kParts);
  double* v = c->mfe_work;        // the Chebyshev vectors are free here
  double* w = c->mfe_work + G.nf;
  double* part = c->mfe_work + 3 * G.nf + G.nc;  // kParts partial results, past every work vector
  double h[kParts];
  const auto reduce = [&](bool is_max) {
    PM_HIP(hipMemcpyAsync(h, part, sizeof(h), hipMemcpyDeviceToHost, s));
    PM_HIP(hipStreamSynchronize(s));
    double m = 0.0;
    for (int i = 0; i < kParts; ++i) m = is_max ? std::max(m, h[i]) : m + h[i];
    return m;
  };
  k_qq_diag<<<blocks_for(G.nf), kBlock, 0, s>>>(G, c->Mq, c->mfe_lq, c->mfe_dqinv, v);
  PM_CHECK_LAUNCH();
  k_max_part<<<kParts, 256, 0, s>>>(G.nf, v, part);
  PM_CHECK_LAUNCH();
  const double gersh = reduce(true);
  // lambda_max(D^-1 A_qq) by power iterations (Gershgorin's bound is loose on
  // distorted cells with anisotropic permeability), capped by Gershgorin
  k_qq_seed<<<blocks_for(G.nf), kBlock, 0, s>>>(G.nf, v);
  k_scale_sumsq_part<<<kParts, 256, 0, s>>>(G.nf, v, 1.0, part);
  PM_CHECK_LAUNCH();
  double nv = std::sqrt(reduce(false)), lam = gersh;
  for (int it = 0; it < 15 && nv > 0.0; ++it) {
    k_scale_sumsq_part<<<kParts, 256, 0, s>>>(G.nf, v, 1.0 / nv, part);  // v /= |v|
    k_qq_dinv_apply<<<blocks_for(G.nf), kBlock, 0, s>>>(G, c->Mq, c->mfe_dqinv, v, w);
    k_scale_sumsq_part<<<kParts, 256, 0, s>>>(G.nf, w, 1.0, part);
    PM_CHECK_LAUNCH();
    nv = std::sqrt(reduce(false));
    lam = nv;  // |D^-1 A v| for |v| = 1
    std::swap(v, w);
  }
  c->mfe_qmax = std::min(gersh, 1.1 * lam);
  c->mfe_valid = true;
}

// z = M^-1 r for M = [[M_uu, 0, 0], [0, M_qq, 0], [A_pu, dt A_pq, M_Cp]]
// (eq. prec), order [u; q; p]: z_u = the A_uu V-cycles (cycles_u, FP64
// levels) on r_u, z_q = kQqChebDegree Chebyshev-Jacobi sweeps on A_qq z_q =
// r_q from zero over [qmax/5, qmax], z_p = the C~_p V-cycles (cycles_pi) on
// r_p - A_pu z_u - dt A_pq z_q.
void apply_btp(pm_ctx* c, const double* r, double* z) {
  const Grid G = grid_of(c);
  hipStream_t s = c->s;
  const int64_t nq = G.nf;
  const double* ru = r;
  const double* rq = r + c->n_u;
  const double* rp = r + c->n_u + nq;
  double* zu = z;
  double* zq = z + c->n_u;
  double* zp = z + c->n_u + nq;
  amg_vcycle(s, c->Hu, ru, zu);
  // Chebyshev sweeps; the result lands in zq (ping-pong through x1)
  double* x1 = c->mfe_work;
  double* dq = c->mfe_work + nq;
  double* tp = c->mfe_work + 3 * nq;
  const double hi = c->mfe_qmax, lo = 0.2 * c->mfe_qmax;
  const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
  double rho = 1.0 / sigma;
  const int deg = kQqChebDegree;
  double* cur = (deg % 2 == 1) ? zq : x1;  // the last step writes zq
  double* nxt = (deg % 2 == 1) ? x1 : zq;
  k_qq_cheb<<<blocks_for(nq), kBlock, 0, s>>>(G, c->Mq, c->mfe_dqinv, rq, nullptr, cur, dq, 0.0, 1.0 / theta, 1);
  PM_CHECK_LAUNCH();
  for (int k = 1; k < deg; ++k) {
    const double rn = 1.0 / (2.0 * sigma - rho);
    const double c1 = rn * rho, c2 = 2.0 * rn / delta;
    rho = rn;
    k_qq_cheb<<<blocks_for(nq), kBlock, 0, s>>>(G, c->Mq, c->mfe_dqinv, rq, cur, nxt, dq, c1, c2, 0);
    PM_CHECK_LAUNCH();
    std::swap(cur, nxt);
  }
  k_btp_p<<<blocks_for(G.nc), kBlock, 0, s>>>(G, c->bc_kind, c->ae, zu, zq, rp, c->dt, tp);
  PM_CHECK_LAUNCH();
  amg_vcycle(s, c->Hcp, tp, zp);
}

// right-hand side [f_u; f_q; f_p] of the MFE step: the traction load, f_q on
// the drained faces, and f_p = A_pu u_prev + S|T| p_prev (+ A_stab p_prev in
// increment form) without the hybrid system's lifting of the face pressures
void build_rhs_mfe(pm_ctx* c, const double* u_prev, const double* p_prev, double* b) {
  const Grid G = grid_of(c);
  // the hybrid right-hand side's u and p rows with a zero face pressure (no lifting)
  const double p_top = c->p_top;
  c->p_top = 0.0;
  try {
    build_rhs(c, u_prev, p_prev, c->rvec);
  } catch (...) {
    c->p_top = p_top;
    throw;
  }
  c->p_top = p_top;
  PM_HIP(hipMemcpyAsync(b, c->rvec, sizeof(double) * c->n_u, hipMemcpyDeviceToDevice, c->s));
  PM_HIP(hipMemcpyAsync(b + c->n_u + G.nf, c->rvec + c->n_u, sizeof(double) * c->n_p, hipMemcpyDeviceToDevice, c->s));
  k_rhs_q_mfe<<<blocks_for(G.nf), kBlock, 0, c->s>>>(G, p_top, b + c->n_u);
  PM_CHECK_LAUNCH();
}

void apply_mfe(pm_ctx* c, const double* x, double* y) {
  const Grid G = grid_of(c);
  ensure_mq(c);
  const int64_t nq = G.nf;
  const double* u = x;
  const double* q = x + c->n_u;
  const double* p = x + c->n_u + nq;
  double* yu = y;
  double* yq = y + c->n_u;
  double* yp = y + c->n_u + nq;
  // u-rows A_uu u + A_up p: the hybrid operator's kernels (the matrix-free
  // stencil on lattices, the sliced ELL level 0 otherwise)
  apply_ah_u(c, u, p, yu);
  k_mfe_q<<<blocks_for(G.nf), kBlock, 0, c->s>>>(G, c->Mq, q, p, yq);
  PM_CHECK_LAUNCH();
  k_mfe_p<<<blocks_for(G.nc), kBlock, 0, c->s>>>(G, c->bc_kind, c->ae, c->vol, c->stabw, u, q, p, c->S, c->dt,
                                                 c->opts.stabilize, yp);
  PM_CHECK_LAUNCH();
}

}  // namespace pm
