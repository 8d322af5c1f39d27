// Finest level of the face-pressure Schur complement, applied cell by cell.
//
// C~_pi = sum_T [ M_T^-1 - (dt / B~_T) g_T g_T^T ] (Sec. 4) is a sum of
// symmetric 6x6 element matrices.  Each is stored once, packed (21 values,
// structure of arrays), and a face row is formed from the (one or two) cells
// that share the face: 21 values per cell instead of 11 stored entries and
// column indices per face, about a third of the bytes of the assembled rows,
// and no index arrays (structured face numbering).  Dirichlet faces (the
// drained top) are identity rows with zero columns, as in the assembled
// matrix.  Coarser levels and the Galerkin products use the assembled matrix.
#include "pm_internal.h"

namespace pm {

void CellPiOp::free_all() {
  dfree(C);
  dfree(C32);
  C = nullptr;
  C32 = nullptr;
  on = false;
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

__device__ inline bool face_of_thread(const Grid& G, int64_t& f) {
  f = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  return f < G.nf;
}

// (C~_pi x)_f over the free columns of the free row f, f at (i,j,k) of
// orientation O.  The packed-matrix entry of each term is a compile-time
// row of C, so every load is a wave-uniform base plus a 32-bit offset.
template <int O, class T>
__device__ __forceinline__ T cpi_row_o(const Grid& G, uint32_t i, uint32_t j, uint32_t k, const T* __restrict__ C,
                                       const T* __restrict__ x) {
  T acc = (T)0;
  const uint32_t top = (uint32_t)G.nz - 1;
  visit_face_cells<O>(G, i, j, k, [&](auto lc, uint32_t c, const uint32_t F[6], uint32_t ck) {
    constexpr int l = decltype(lc)::value;
#pragma unroll
    for (int e = 0; e < 6; ++e) {
      const T v = ld32(C + (size_t)sym6(l < e ? l : e, l < e ? e : l) * G.nc, c) * ld32(x, F[e]);
      if (e != 5 || ck != top) acc += v;  // the top face of the top layer is a zero column
    }
  });
  return acc;
}

template <class T>
__device__ __forceinline__ T cpi_cells_row(const Grid& G, int64_t f, const T* __restrict__ C,
                                           const T* __restrict__ x) {
  uint32_t i, j, k;
  const int o = face_pos(G, (uint32_t)f, i, j, k);
  if (o == 0) return cpi_row_o<0, T>(G, i, j, k, C, x);
  if (o == 1) return cpi_row_o<1, T>(G, i, j, k, C, x);
  return cpi_row_o<2, T>(G, i, j, k, C, x);
}

template <class T>
__global__ void __launch_bounds__(256) k_cp_cheb(Grid G, const T* __restrict__ C, const T* __restrict__ dinv,
                                                 const T* __restrict__ b, const T* __restrict__ xin,
                                                 T* __restrict__ xout, T* __restrict__ d, T c1, T c2) {
  int64_t f;
  if (!face_of_thread(G, f)) return;
  const T ax = pi_fixed(G, f) ? xin[f] : cpi_cells_row<T>(G, f, C, xin);
  const T z = dinv[f] * (b[f] - ax);
  const T dn = c1 * d[f] + c2 * z;
  d[f] = dn;
  xout[f] = xin[f] + dn;
}

template <class T>
__global__ void __launch_bounds__(256) k_cp_residual(Grid G, const T* __restrict__ C, const T* __restrict__ b,
                                                     const T* __restrict__ x, T* __restrict__ r) {
  int64_t f;
  if (!face_of_thread(G, f)) return;
  const T ax = pi_fixed(G, f) ? x[f] : cpi_cells_row<T>(G, f, C, x);
  r[f] = b[f] - ax;
}

__global__ void __launch_bounds__(256) k_cp_apply(Grid G, const double* __restrict__ C,
                                                  const double* __restrict__ x, double* __restrict__ y) {
  int64_t f;
  if (!face_of_thread(G, f)) return;
  y[f] = pi_fixed(G, f) ? x[f] : cpi_cells_row<double>(G, f, C, x);
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
  if (!op.C) op.C = dalloc<double>(21 * G.nc);
  if (c->opts.precond_fp32 && !op.C32) op.C32 = dalloc<float>(21 * G.nc);
  k_cpi_cells<<<blocks_for(G.nc), kBlock, 0, s>>>(G, c->Minv, c->g, c->bp, c->dt, op.C,
                                                     c->opts.precond_fp32 ? op.C32 : nullptr);
  PM_CHECK_LAUNCH();
  op.on = true;
}

template <class T>
void cellpi_cheb_step(hipStream_t s, const Grid& G, const CellPiOp& op, const T* dinv, const T* b, const T* xin,
                      T* xout, T* d, T c1, T c2) {
  k_cp_cheb<T><<<blocks_for(G.nf), kBlock, 0, s>>>(G, cp_C<T>(op), dinv, b, xin, xout, d, c1, c2);
  PM_CHECK_LAUNCH();
}
template void cellpi_cheb_step<double>(hipStream_t, const Grid&, const CellPiOp&, const double*, const double*,
                                       const double*, double*, double*, double, double);
template void cellpi_cheb_step<float>(hipStream_t, const Grid&, const CellPiOp&, const float*, const float*,
                                      const float*, float*, float*, float, float);

template <class T>
void cellpi_residual(hipStream_t s, const Grid& G, const CellPiOp& op, const T* b, const T* x, T* r) {
  k_cp_residual<T><<<blocks_for(G.nf), kBlock, 0, s>>>(G, cp_C<T>(op), b, x, r);
  PM_CHECK_LAUNCH();
}
template void cellpi_residual<double>(hipStream_t, const Grid&, const CellPiOp&, const double*, const double*,
                                      double*);
template void cellpi_residual<float>(hipStream_t, const Grid&, const CellPiOp&, const float*, const float*,
                                     float*);

void cellpi_apply(hipStream_t s, const Grid& G, const CellPiOp& op, const double* x, double* y) {
  k_cp_apply<<<blocks_for(G.nf), kBlock, 0, s>>>(G, op.C, x, y);
  PM_CHECK_LAUNCH();
}

}  // namespace pm
