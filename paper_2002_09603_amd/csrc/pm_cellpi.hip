// Finest level of the face-pressure Schur complement, applied cell by cell.
//
// C~_pi = sum_T [ M_T^-1 - (dt / B~_T) g_T g_T^T ] (Sec. 4) is a sum of
// symmetric 6x6 element matrices.  Each is stored once, packed (21 values,
// structure of arrays), and a face row is formed from the (one or two) cells
// that share the face: 21 values per cell instead of 11 stored entries and
// column indices per face, about a third of the bytes of the assembled rows,
// and no index arrays (structured face numbering).  When M_T^-1 couples only
// the two faces of each direction (axis-aligned boxes, diagonal
// permeability) the element matrix is kept as its 9 block entries and
// dt / B~_T, 10 values per cell, and the rank-one term is formed on the fly
// (g = M^-1 1 from the blocks).  Dirichlet faces (the drained top) are
// identity rows with zero columns, as in the assembled matrix.  Coarser
// levels and the Galerkin products use the assembled matrix.
#include "pm_internal.h"

namespace pm {

void CellPiOp::free_all() {
  dfree(C);
  dfree(C32);
  C = nullptr;
  C32 = nullptr;
  on = false;
  block = false;
  nvals = 0;
}

namespace {

__global__ void k_cpi_cells(Grid G, const double* __restrict__ Minv, const double* __restrict__ gv,
                            const double* __restrict__ bp, double dt, double* __restrict__ C,
                            float* __restrict__ C32) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= G.nc) return;
  const double sc = dt / bp[c];
  double g[6];
  for (int a = 0; a < 6; ++a) g[a] = gv[(size_t)a * G.nc + c];
  for (int a = 0; a < 6; ++a)
    for (int b = a; b < 6; ++b) {
      const double v = Minv[(size_t)(a * 6 + b) * G.nc + c] - sc * g[a] * g[b];
      const size_t q = (size_t)sym6(a, b) * G.nc + c;
      C[q] = v;
      if (C32) C32[q] = (float)v;
    }
}

// block form: the direction blocks of M_T^-1 ([3d] (2d,2d), [3d+1] (2d,2d+1),
// [3d+2] (2d+1,2d+1)) and dt / B~_T
__global__ void k_cpi_cells_block_minv(Grid G, const double* __restrict__ Minv, const double* __restrict__ bp,
                                       double dt, double* __restrict__ C, float* __restrict__ C32) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= G.nc) return;
  double v[10];
  for (int d = 0; d < 3; ++d) {
    const int a = 2 * d, b = 2 * d + 1;
    v[3 * d + 0] = Minv[(size_t)(a * 6 + a) * G.nc + c];
    v[3 * d + 1] = 0.5 * (Minv[(size_t)(a * 6 + b) * G.nc + c] + Minv[(size_t)(b * 6 + a) * G.nc + c]);
    v[3 * d + 2] = Minv[(size_t)(b * 6 + b) * G.nc + c];
  }
  v[9] = dt / bp[c];
  for (int q = 0; q < 10; ++q) {
    C[(size_t)q * G.nc + c] = v[q];
    if (C32) C32[(size_t)q * G.nc + c] = (float)v[q];
  }
}

__device__ inline bool cell_of_thread(const Grid& G, uint32_t& i, uint32_t& j, uint32_t& k) {
  const int64_t c = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (c >= G.nc) return false;
  int a, b, e;
  G.cell_ijk(c, a, b, e);
  i = (uint32_t)a;
  j = (uint32_t)b;
  k = (uint32_t)e;
  return true;
}

// sum_e C_T[l, e] x[F_T[e]] over the free columns, l a compile-time local face
template <class T>
struct CpiTerm {
  const Grid& G;
  const T* __restrict__ C;
  const T* __restrict__ x;
  template <int L>
  __device__ __forceinline__ T operator()(LocalFace<L>, uint32_t c, const uint32_t F[6], uint32_t ck) const {
    T acc = (T)0;
#pragma unroll
    for (int e = 0; e < 6; ++e) {
      const T v = ld32(C + (size_t)sym6(L < e ? L : e, L < e ? e : L) * G.nc, c) * ld32(x, F[e]);
      if (!pi_fixed_local(G, (int)ck, e)) acc += v;  // a drained top face is a zero column
    }
    return acc;
  }
};

// the same from the block form: row L = 2d + s of
// M^-1 - sc g g^T is the block row [m_L,2d, m_L,2d+1] on faces 2d, 2d+1
// minus sc g_L (g^T x), g^T x over the free faces of the cell
template <class T>
struct CpiBlockTerm {
  const Grid& G;
  const T* __restrict__ C;
  const T* __restrict__ x;
  template <int L>
  __device__ __forceinline__ T operator()(LocalFace<L>, uint32_t c, const uint32_t F[6], uint32_t ck) const {
    constexpr int d = L >> 1, sd = L & 1;
    T m[9], xv[6];
#pragma unroll
    for (int q = 0; q < 9; ++q) m[q] = ld32(C + (size_t)q * G.nc, c);
    const T sc = ld32(C + (size_t)9 * G.nc, c);
#pragma unroll
    for (int e = 0; e < 6; ++e) xv[e] = ld32(x, F[e]);
    if (pi_fixed_local(G, (int)ck, 5)) xv[5] = (T)0;  // a drained top face is a zero column
    T gx = (T)0;
#pragma unroll
    for (int a = 0; a < 3; ++a) gx += (m[3 * a] + m[3 * a + 1]) * xv[2 * a] + (m[3 * a + 1] + m[3 * a + 2]) * xv[2 * a + 1];
    const T md = m[3 * d + 2 * sd], mo = m[3 * d + 1];
    const T gl = md + mo;
    return (sd ? mo : md) * xv[2 * d] + (sd ? md : mo) * xv[2 * d + 1] - sc * gl * gx;
  }
};

template <class T, bool BLOCK>
using CpiTermOf = typename std::conditional<BLOCK, CpiBlockTerm<T>, CpiTerm<T>>::type;

// Chebyshev step on the finest C~_pi level, one thread per cell (its owned faces)
template <class T, bool BLOCK>
__global__ void __launch_bounds__(256) k_cp_cheb(Grid G, const T* __restrict__ C, const T* __restrict__ dinv,
                                                 const T* __restrict__ b, const T* __restrict__ xin,
                                                 T* __restrict__ xout, T* __restrict__ d, T c1, T c2) {
  uint32_t i, j, k;
  if (!cell_of_thread(G, i, j, k)) return;
  owned_face_rows<T>(G, i, j, k, CpiTermOf<T, BLOCK>{G, C, xin}, [&](uint32_t f, bool fixed, T acc) {
    const T ax = fixed ? xin[f] : acc;
    const T z = dinv[f] * (b[f] - ax);
    const T dn = c1 * d[f] + c2 * z;
    d[f] = dn;
    xout[f] = xin[f] + dn;
  });
}

template <class T, bool BLOCK>
__global__ void __launch_bounds__(256) k_cp_residual(Grid G, const T* __restrict__ C, const T* __restrict__ b,
                                                     const T* __restrict__ x, T* __restrict__ r) {
  uint32_t i, j, k;
  if (!cell_of_thread(G, i, j, k)) return;
  owned_face_rows<T>(G, i, j, k, CpiTermOf<T, BLOCK>{G, C, x},
                     [&](uint32_t f, bool fixed, T acc) { r[f] = b[f] - (fixed ? x[f] : acc); });
}

template <class T, bool BLOCK>
__global__ void __launch_bounds__(256) k_cp_apply(Grid G, const T* __restrict__ C, const T* __restrict__ x,
                                                  T* __restrict__ y) {
  uint32_t i, j, k;
  if (!cell_of_thread(G, i, j, k)) return;
  owned_face_rows<T>(G, i, j, k, CpiTermOf<T, BLOCK>{G, C, x},
                     [&](uint32_t f, bool fixed, T acc) { y[f] = fixed ? x[f] : acc; });
}

template <class T>
const T* cp_C(const CellPiOp& op);
template <>
const double* cp_C<double>(const CellPiOp& op) { return op.C; }
template <>
const float* cp_C<float>(const CellPiOp& op) { return op.C32; }

}  // namespace

void cellpi_build(pm_ctx* c, hipStream_t s) {
  CellPiOp& op = c->cpi;
  const Grid G = grid_of(c);
  const int nv = c->mblock ? 10 : 21;
  if (op.nvals != nv) {
    dfree(op.C);
    dfree(op.C32);
    op.C = nullptr;
    op.C32 = nullptr;
    op.nvals = nv;
  }
  if (!op.C) op.C = dalloc<double>((int64_t)nv * G.nc);
  if (c->opts.precond_fp32 && !op.C32) op.C32 = dalloc<float>((int64_t)nv * G.nc);
  op.block = c->mblock;
  if (op.block) {
    // the block entries straight from M^-1 (c->Mb is packed on the other stream)
    k_cpi_cells_block_minv<<<blocks_for(G.nc), kBlock, 0, s>>>(G, c->Minv, c->bp, c->dt, op.C,
                                                                  c->opts.precond_fp32 ? op.C32 : nullptr);
  } else {
    k_cpi_cells<<<blocks_for(G.nc), kBlock, 0, s>>>(G, c->Minv, c->g, c->bp, c->dt, op.C,
                                                       c->opts.precond_fp32 ? op.C32 : nullptr);
  }
  PM_CHECK_LAUNCH();
  op.on = true;
}

template <class T>
void cellpi_cheb_step(hipStream_t s, const Grid& G, const CellPiOp& op, const T* dinv, const T* b, const T* xin,
                      T* xout, T* d, T c1, T c2) {
  if (op.block)
    k_cp_cheb<T, true><<<blocks_for(G.nc), kBlock, 0, s>>>(G, cp_C<T>(op), dinv, b, xin, xout, d, c1, c2);
  else
    k_cp_cheb<T, false><<<blocks_for(G.nc), kBlock, 0, s>>>(G, cp_C<T>(op), dinv, b, xin, xout, d, c1, c2);
  PM_CHECK_LAUNCH();
}
template void cellpi_cheb_step<double>(hipStream_t, const Grid&, const CellPiOp&, const double*, const double*,
                                       const double*, double*, double*, double, double);
template void cellpi_cheb_step<float>(hipStream_t, const Grid&, const CellPiOp&, const float*, const float*,
                                      const float*, float*, float*, float, float);

template <class T>
void cellpi_residual(hipStream_t s, const Grid& G, const CellPiOp& op, const T* b, const T* x, T* r) {
  if (op.block)
    k_cp_residual<T, true><<<blocks_for(G.nc), kBlock, 0, s>>>(G, cp_C<T>(op), b, x, r);
  else
    k_cp_residual<T, false><<<blocks_for(G.nc), kBlock, 0, s>>>(G, cp_C<T>(op), b, x, r);
  PM_CHECK_LAUNCH();
}
template void cellpi_residual<double>(hipStream_t, const Grid&, const CellPiOp&, const double*, const double*,
                                      double*);
template void cellpi_residual<float>(hipStream_t, const Grid&, const CellPiOp&, const float*, const float*,
                                     float*);

template <class T>
void cellpi_apply_t(hipStream_t s, const Grid& G, const CellPiOp& op, const T* x, T* y) {
  if (op.block)
    k_cp_apply<T, true><<<blocks_for(G.nc), kBlock, 0, s>>>(G, cp_C<T>(op), x, y);
  else
    k_cp_apply<T, false><<<blocks_for(G.nc), kBlock, 0, s>>>(G, cp_C<T>(op), x, y);
  PM_CHECK_LAUNCH();
}
void cellpi_apply(hipStream_t s, const Grid& G, const CellPiOp& op, const double* x, double* y) {
  cellpi_apply_t<double>(s, G, op, x, y);
}
void cellpi_apply(hipStream_t s, const Grid& G, const CellPiOp& op, const float* x, float* y) {
  cellpi_apply_t<float>(s, G, op, x, y);
}

}  // namespace pm
