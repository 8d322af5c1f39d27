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

// y_u += A_up p on the free displacement dofs (y_u holds A_uu u)
__global__ void __launch_bounds__(256) k_mfe_up(Grid G, int kind, const double* __restrict__ ae,
                                                const double* __restrict__ p, double* __restrict__ yu) {
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
        for (int d = 0; d < 3; ++d) cp[d] += ae[(size_t)(3 * a + d) * G.nc + c] * p[c];
      }
  for (int d = 0; d < 3; ++d)
    if (!u_fixed(G, kind, i, j, k, d)) yu[3 * n + d] += cp[d];
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
  double* Lq = dalloc<double>(G.nf);
  k_cp_lump<<<blocks_for(G.nf), kBlock, 0, s>>>(G, c->Mq, Lq);
  PM_CHECK_LAUNCH();
  k_cp_fill<<<blocks_for(G.nc), kBlock, 0, s>>>(G, Lq, c->bp, c->alpha, c->stabw, c->dt, c->opts.stabilize,
                                                c->Cp.rowptr, c->Cp.col, c->Cp.val);
  PM_CHECK_LAUNCH();
  dfree(Lq);
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
  apply_csr(c, c->Auu, u, yu);
  k_mfe_up<<<blocks_for(G.nn), kBlock, 0, c->s>>>(G, c->bc_kind, c->ae, p, yu);
  PM_CHECK_LAUNCH();
  k_mfe_q<<<blocks_for(G.nf), kBlock, 0, c->s>>>(G, c->Mq, q, p, yq);
  PM_CHECK_LAUNCH();
  k_mfe_p<<<blocks_for(G.nc), kBlock, 0, c->s>>>(G, c->bc_kind, c->ae, c->vol, c->stabw, u, q, p, c->S, c->dt,
                                                 c->opts.stabilize, yp);
  PM_CHECK_LAUNCH();
}

}  // namespace pm
