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
      if (e != 5 || ck != (uint32_t)G.nz - 1) acc += v;  // the top face of the top layer is a zero column
    }
    return acc;
  }
};

// Chebyshev step on the finest C~_pi level, one thread per cell (its owned faces)
template <class T>
__global__ void __launch_bounds__(256) k_cp_cheb(Grid G, const T* __restrict__ C, const T* __restrict__ dinv,
                                                 const T* __restrict__ b, const T* __restrict__ xin,
                                                 T* __restrict__ xout, T* __restrict__ d, T c1, T c2) {
  uint32_t i, j, k;
  if (!cell_of_thread(G, i, j, k)) return;
  owned_face_rows<T>(G, i, j, k, CpiTerm<T>{G, C, xin}, [&](uint32_t f, bool fixed, T acc) {
    const T ax = fixed ? xin[f] : acc;
    const T z = dinv[f] * (b[f] - ax);
    const T dn = c1 * d[f] + c2 * z;
    d[f] = dn;
    xout[f] = xin[f] + dn;
  });
}

template <class T>
__global__ void __launch_bounds__(256) k_cp_residual(Grid G, const T* __restrict__ C, const T* __restrict__ b,
                                                     const T* __restrict__ x, T* __restrict__ r) {
  uint32_t i, j, k;
  if (!cell_of_thread(G, i, j, k)) return;
  owned_face_rows<T>(G, i, j, k, CpiTerm<T>{G, C, x},
                     [&](uint32_t f, bool fixed, T acc) { r[f] = b[f] - (fixed ? x[f] : acc); });
}

__global__ void __launch_bounds__(256) k_cp_apply(Grid G, const double* __restrict__ C,
                                                  const double* __restrict__ x, double* __restrict__ y) {
  uint32_t i, j, k;
  if (!cell_of_thread(G, i, j, k)) return;
  owned_face_rows<double>(G, i, j, k, CpiTerm<double>{G, C, x},
                          [&](uint32_t f, bool fixed, double acc) { y[f] = fixed ? x[f] : acc; });
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
  k_cp_cheb<T><<<blocks_for(G.nc), kBlock, 0, s>>>(G, cp_C<T>(op), dinv, b, xin, xout, d, c1, c2);
  PM_CHECK_LAUNCH();
}
template void cellpi_cheb_step<double>(hipStream_t, const Grid&, const CellPiOp&, const double*, const double*,
                                       const double*, double*, double*, double, double);
template void cellpi_cheb_step<float>(hipStream_t, const Grid&, const CellPiOp&, const float*, const float*,
                                      const float*, float*, float*, float, float);

template <class T>
void cellpi_residual(hipStream_t s, const Grid& G, const CellPiOp& op, const T* b, const T* x, T* r) {
  k_cp_residual<T><<<blocks_for(G.nc), kBlock, 0, s>>>(G, cp_C<T>(op), b, x, r);
  PM_CHECK_LAUNCH();
}
template void cellpi_residual<double>(hipStream_t, const Grid&, const CellPiOp&, const double*, const double*,
                                      double*);
template void cellpi_residual<float>(hipStream_t, const Grid&, const CellPiOp&, const float*, const float*,
                                     float*);

void cellpi_apply(hipStream_t s, const Grid& G, const CellPiOp& op, const double* x, double* y) {
  k_cp_apply<<<blocks_for(G.nc), kBlock, 0, s>>>(G, op.C, x, y);
  PM_CHECK_LAUNCH();
}

}  // namespace pm
