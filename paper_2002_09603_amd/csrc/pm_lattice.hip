// Finest-level displacement operator on lattice meshes.
//
// When the cells are translates of one parallelepiped (uniform boxes, as in
// the paper's cantilever and reservoir grids), the Q1 element stiffness of
// cell T is E_T Khat with one 24x24 matrix Khat for unit modulus (nu is
// uniform), and the coupling column a_T is one vector ahat.  A row of A_uu is
// then a sum over the (up to 8) cells around the node of E_T times 3 rows of
// Khat applied to the 8 nodal displacements of the cell: 576 multiply-adds
// per node, with Khat and ahat read at wave-uniform addresses (scalar loads)
// and only the vectors, E and the smoother's diagonal blocks streamed from
// memory.  This replaces reading the assembled 27-block rows (76 B per block
// in FP64, 40 B in FP32) on the level where they dominate the V-cycle and the
// Krylov operator.  Dirichlet rows and columns follow u_fixed, exactly as the
// assembled matrix does (identity rows, zero columns).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>

#include "pm_internal.h"

namespace pm {

void LatticeOp::free_all() {
  dfree(Kh);
  dfree(Kh32);
  dfree(ah);
  dfree(E32);
  Kh = nullptr;
  Kh32 = nullptr;
  ah = nullptr;
  E32 = nullptr;
  E = nullptr;
  on = false;
  sym = false;
  cube = false;
}

namespace {

__device__ inline bool node_of_thread(const Grid& G, int64_t& n, int& i, int& j, int& k) {
  n = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (n >= G.nn) return false;
  // plain 32-bit division here (fewer registers live across the stencil than
  // the multiply-shift form)
  const uint32_t nx1 = (uint32_t)G.nx + 1, ny1 = (uint32_t)G.ny + 1;
  const uint32_t m = (uint32_t)n;
  const uint32_t r = m / nx1;
  i = (int)(m - r * nx1);
  k = (int)(r / ny1);
  j = (int)(r - (uint32_t)k * ny1);
  return true;
}

// The clamped 3x3x3 node box and 2x2x2 cell box around node (i,j,k): the
// lower-corner node and cell plus non-negative offsets per axis, all in 32
// bits (the lattice is used only while 3 n_n doubles stay below 4 GiB), so a
// neighbour is addressed as the kernel's base pointer plus one 32-bit byte
// offset.  A neighbour outside the mesh is clamped onto the node itself; it
// only belongs to cells outside the mesh, whose modulus is taken as zero.
// explicit fused multiply-add: with entries of Khat repeated (box cells) the
// compiler would otherwise share products between sums and split the FMAs
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

// The 24x24 unit stiffness as read by the stencil: KDense reads all 576
// entries, KSym rebuilds them from the 48 values of a box cell.
template <class T>
struct KDense {
  const T* __restrict__ p;
  __device__ __forceinline__ T operator()(int a, int b, int r, int c) const { return p[(3 * a + r) * 24 + 3 * b + c]; }
};
template <class T>
struct KSym {
  T k[48];
  __device__ __forceinline__ T operator()(int a, int b, int r, int c) const {
    const T v = k[6 * (a ^ b) + sym_slot(r, c)];
    return sym_negated(a, b, r, c) ? -v : v;
  }
};

template <class T>
struct KCube {
  T k[12];
  __device__ __forceinline__ T operator()(int a, int b, int r, int c) const {
    const int d = a ^ b, lo = r < c ? r : c, hi = r < c ? c : r;
    const T v = k[cube_slot(d, lo, hi)];
    return (sym_negated(a, b, r, c) != cube_negated(d, lo, hi)) ? -v : v;
  }
};

struct Box {
  uint32_t nxo[3], nyo[3], nzo[3];  // byte offsets of the lower/middle/upper neighbour node
  uint32_t cxo, cyo, czo;           // cell offset of the upper cell along each axis
  bool inx[2], iny[2], inz[2];      // lower/upper cell inside the mesh
  uint32_t n0, c0;                  // lower-corner node (byte offset) and cell (index)
};

// node offsets in bytes for vectors of TX (3 per node); the strides are
// wave-uniform, so each offset is a select rather than a multiply
template <class TX>
__device__ __forceinline__ Box box_of(const Grid& G, int64_t n, int i, int j, int k) {
  constexpr uint32_t kNode = 3 * sizeof(TX);
  Box B;
  const uint32_t sy = ((uint32_t)G.nx + 1) * kNode, sz = sy * ((uint32_t)G.ny + 1);
  const bool lx = i > 0, ly = j > 0, lz = k > 0;
  const bool hx = i < G.nx, hy = j < G.ny, hz = k < G.nz;
  B.nxo[0] = 0;
  B.nxo[1] = lx ? kNode : 0u;
  B.nxo[2] = B.nxo[1] + (hx ? kNode : 0u);
  B.nyo[0] = 0;
  B.nyo[1] = ly ? sy : 0u;
  B.nyo[2] = B.nyo[1] + (hy ? sy : 0u);
  B.nzo[0] = 0;
  B.nzo[1] = lz ? sz : 0u;
  B.nzo[2] = B.nzo[1] + (hz ? sz : 0u);
  B.n0 = (uint32_t)n * kNode - (B.nxo[1] + B.nyo[1] + B.nzo[1]);
  // cells i-1 and i along x, clamped into [0, nx-1] (nx >= 1)
  B.cxo = (lx && hx) ? 1u : 0u;
  B.cyo = (ly && hy) ? (uint32_t)G.nx : 0u;
  B.czo = (lz && hz) ? (uint32_t)G.nx * (uint32_t)G.ny : 0u;
  B.c0 = (uint32_t)G.cell(i - (int)lx, j - (int)ly, k - (int)lz);
  B.inx[0] = lx;
  B.inx[1] = hx;
  B.iny[0] = ly;
  B.iny[1] = hy;
  B.inz[0] = lz;
  B.inz[1] = hz;
  return B;
}

// a 32-bit byte offset from a wave-uniform base (one VGPR offset per load
// instead of a 64-bit address; constant offsets from it become immediates)
template <class V>
__device__ __forceinline__ const V* at_byte(const V* __restrict__ base, uint32_t off) {
  return reinterpret_cast<const V*>(reinterpret_cast<const char*>(base) + off);
}

// One plane dz of the 3x3 neighbour displacements of node (i,j,k).  MASK
// zeroes Dirichlet components (zero columns of A_uu).
template <class T, class TX, bool MASK>
__device__ __forceinline__ void load_plane(const Grid& G, int kind, const TX* __restrict__ x, const Box& B, int dz,
                                           int i, int j, int k, T u[9][3]) {
#pragma unroll
  for (int dy = 0; dy < 3; ++dy) {
    const uint32_t row = B.n0 + B.nyo[dy] + B.nzo[dz];
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) {
      const uint32_t off = row + B.nxo[dx];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T v = (T)at_byte(x, off)[c];
        u[dx + 3 * dy][c] = (MASK && u_fixed(G, kind, i + dx - 1, j + dy - 1, k + dz - 1, c)) ? (T)0 : v;
      }
    }
  }
}

// acc += contributions of the 4 cells of layer oz around the node; lo and hi
// are the neighbour planes below and above that cell layer
template <class T, class KS>
__device__ __forceinline__ void cell_layer(const KS& Kh, const T* __restrict__ E, const Box& B,
                                           const T lo[9][3], const T hi[9][3], int oz, T acc[3]) {
#pragma unroll
  for (int oy = 0; oy < 2; ++oy)
#pragma unroll
    for (int ox = 0; ox < 2; ++ox) {
      const bool in = B.inz[oz] && B.iny[oy] && B.inx[ox];
      const T ev = *at_byte(E, (B.c0 + (ox ? B.cxo : 0u) + (oy ? B.cyo : 0u) + (oz ? B.czo : 0u)) *
                                  (uint32_t)sizeof(T));
      const T e = in ? ev : (T)0;
      const int a = (1 - ox) + 2 * (1 - oy) + 4 * (1 - oz);
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        T sum = (T)0;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
          const int q = (ox + (b & 1)) + 3 * (oy + ((b >> 1) & 1));
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const T uv = ((b >> 2) & 1) ? hi[q][c] : lo[q][c];
            sum = fmadd(Kh(a, b, r, c), uv, sum);
          }
        }
        acc[r] += e * sum;
      }
    }
}

// acc = sum over the cells T around node (i,j,k) of E_T Khat[3a..3a+2, :] u_T,
// the neighbour planes loaded one at a time
template <class T, class TX, bool MASK, class KS>
__device__ __forceinline__ void lattice_rows(const Grid& G, int kind, const KS& Kh,
                                             const T* __restrict__ E, const TX* __restrict__ x, const Box& B, int i,
                                             int j, int k, T acc[3]) {
  acc[0] = acc[1] = acc[2] = (T)0;
  T pa[9][3], pb[9][3];
  load_plane<T, TX, MASK>(G, kind, x, B, 0, i, j, k, pa);
  load_plane<T, TX, MASK>(G, kind, x, B, 1, i, j, k, pb);
  cell_layer<T, KS>(Kh, E, B, pa, pb, 0, acc);
  load_plane<T, TX, MASK>(G, kind, x, B, 2, i, j, k, pa);
  cell_layer<T, KS>(Kh, E, B, pb, pa, 1, acc);
}

// no Dirichlet component among the 27 neighbours of node (i,j,k)
__device__ inline bool free_neighbourhood(const Grid& G, int kind, int i, int j, int k) {
  if (kind == PM_BC_CANTILEVER) return i >= 2;
  if (k < 2) return false;
  if (kind != PM_BC_ROLLERS) return true;
  return i >= 2 && i <= G.nx - 2 && j >= 2 && j <= G.ny - 2;
}

// (A x) at node n: Dirichlet rows are identity
template <class T, class KS>
__device__ __forceinline__ void lattice_Ax(const Grid& G, int kind, const KS& Kh,
                                           const T* __restrict__ E, const T* __restrict__ x, int64_t n, int i, int j,
                                           int k, T ax[3]) {
  const Box B = box_of<T>(G, n, i, j, k);
  if (free_neighbourhood(G, kind, i, j, k))
    lattice_rows<T, T, false, KS>(G, kind, Kh, E, x, B, i, j, k, ax);
  else
    lattice_rows<T, T, true, KS>(G, kind, Kh, E, x, B, i, j, k, ax);
#pragma unroll
  for (int a = 0; a < 3; ++a)
    if (u_fixed(G, kind, i, j, k, a)) ax[a] = x[3 * n + a];
}

// Minimum waves per SIMD for the stencil kernels.  In FP64 the neighbour
// planes in flight take about 170 vector registers, one over the limit for
// three resident waves; capping the allocation there costs a few spilled
// values and runs faster than two waves.  In FP32 the cap at 96 registers
// (five waves) spills a few values and runs about 6% faster than four waves.
template <class T>
constexpr int kLatWaves = sizeof(T) == 8 ? 3 : 5;

template <class T, int KIND, class KS>
__global__ void __launch_bounds__(256, kLatWaves<T>) k_lat_cheb(Grid G, const KS Kh,
                                                  const T* __restrict__ E, const T* __restrict__ dinv,
                                                  const T* __restrict__ b, const T* __restrict__ xin,
                                                  T* __restrict__ xout, T* __restrict__ d, T c1, T c2) {
  int64_t n;
  int i, j, k;
  if (!node_of_thread(G, n, i, j, k)) return;
  T ax[3];
  lattice_Ax<T, KS>(G, KIND, Kh, E, xin, n, i, j, k, ax);
  T res[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) res[a] = b[3 * n + a] - ax[a];
  const T* D = dinv + 9 * n;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const T z = D[3 * a] * res[0] + D[3 * a + 1] * res[1] + D[3 * a + 2] * res[2];
    const int64_t q = 3 * n + a;
    const T dn = c1 * d[q] + c2 * z;
    d[q] = dn;
    xout[q] = xin[q] + dn;
  }
}

template <class T, int KIND, class KS>
__global__ void __launch_bounds__(256, kLatWaves<T>) k_lat_residual(Grid G, const KS Kh,
                                                      const T* __restrict__ E, const T* __restrict__ b,
                                                      const T* __restrict__ x, T* __restrict__ r) {
  int64_t n;
  int i, j, k;
  if (!node_of_thread(G, n, i, j, k)) return;
  T ax[3];
  lattice_Ax<T, KS>(G, KIND, Kh, E, x, n, i, j, k, ax);
#pragma unroll
  for (int a = 0; a < 3; ++a) r[3 * n + a] = b[3 * n + a] - ax[a];
}

template <class T, int KIND, class KS>
__global__ void __launch_bounds__(256, kLatWaves<T>) k_lat_apply(Grid G, const KS Kh, const T* __restrict__ E,
                                                              const T* __restrict__ x, T* __restrict__ y) {
  int64_t n;
  int i, j, k;
  if (!node_of_thread(G, n, i, j, k)) return;
  T ax[3];
  lattice_Ax<T, KS>(G, KIND, Kh, E, x, n, i, j, k, ax);
#pragma unroll
  for (int a = 0; a < 3; ++a) y[3 * n + a] = ax[a];
}

// u-rows of A_H (sgn = +1) or A_H^T (sgn = -1): A_uu u + sgn A_up p on free
// rows, in FP64 from FP64 or FP32 inputs
template <class TX, int KIND, class KS>
__global__ void __launch_bounds__(256, kLatWaves<double>) k_lat_ah_u(Grid G, const KS Kh,
                                                  const double* __restrict__ ah, const double* __restrict__ E,
                                                  const TX* __restrict__ u, const TX* __restrict__ p, double sgn,
                                                  double* __restrict__ y) {
  constexpr int kind = KIND;
  int64_t n;
  int i, j, k;
  if (!node_of_thread(G, n, i, j, k)) return;
  double acc[3];
  const Box B = box_of<TX>(G, n, i, j, k);
  if (free_neighbourhood(G, kind, i, j, k))
    lattice_rows<double, TX, false, KS>(G, kind, Kh, E, u, B, i, j, k, acc);
  else
    lattice_rows<double, TX, true, KS>(G, kind, Kh, E, u, B, i, j, k, acc);
  double cp[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int oz = 0; oz < 2; ++oz)
#pragma unroll
    for (int oy = 0; oy < 2; ++oy)
#pragma unroll
      for (int ox = 0; ox < 2; ++ox) {
        const bool in = B.inz[oz] && B.iny[oy] && B.inx[ox];
        const double pv =
            (double)*at_byte(p, (B.c0 + (ox ? B.cxo : 0u) + (oy ? B.cyo : 0u) + (oz ? B.czo : 0u)) * (uint32_t)sizeof(TX));
        const double pc = in ? pv : 0.0;
        const int a = (1 - ox) + 2 * (1 - oy) + 4 * (1 - oz);
#pragma unroll
        for (int d = 0; d < 3; ++d) cp[d] += ah[3 * a + d] * pc;
      }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int64_t q = 3 * n + d;
    y[q] = u_fixed(G, kind, i, j, k, d) ? (double)u[q] : acc[d] + sgn * cp[d];
  }
}

__global__ void __launch_bounds__(256) k_lat_dev(Grid G, const double* __restrict__ X,
                                                 unsigned long long* __restrict__ out) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double dev = 0.0;
  if (n < G.nn) {
    int i, j, k;
    G.node_ijk(n, i, j, k);
    const int64_t n1 = G.node(G.nx > 0 ? 1 : 0, 0, 0), n2 = G.node(0, G.ny > 0 ? 1 : 0, 0),
                  n3 = G.node(0, 0, G.nz > 0 ? 1 : 0);
    for (int c = 0; c < 3; ++c) {
      const double x0 = X[c];
      const double pred = x0 + i * (X[3 * n1 + c] - x0) + j * (X[3 * n2 + c] - x0) + k * (X[3 * n3 + c] - x0);
      dev = fmax(dev, fabs(X[3 * n + c] - pred));
    }
  }
  __shared__ double sh[256];
  sh[threadIdx.x] = dev;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  // non-negative doubles order like their bit patterns
  if (threadIdx.x == 0) atomicMax(out, (unsigned long long)__double_as_longlong(sh[0]));
}

__global__ void k_lat_to_float(int64_t n, const double* __restrict__ a, float* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

template <class T>
const T* lat_K(const LatticeOp& op);
template <>
const double* lat_K<double>(const LatticeOp& op) { return op.Kh; }
template <>
const float* lat_K<float>(const LatticeOp& op) { return op.Kh32; }
template <class T>
const T* lat_E(const LatticeOp& op);
template <>
const double* lat_E<double>(const LatticeOp& op) { return op.E; }
template <>
const float* lat_E<float>(const LatticeOp& op) { return op.E32; }

// the stencil kernels are instantiated per boundary-condition kind, so each
// carries only its own Dirichlet tests (fewer registers than a run-time kind)
template <class F>
void with_bc_kind(int kind, F&& f) {
  if (kind == PM_BC_CANTILEVER)
    f(std::integral_constant<int, PM_BC_CANTILEVER>{});
  else if (kind == PM_BC_ROLLERS)
    f(std::integral_constant<int, PM_BC_ROLLERS>{});
  else
    f(std::integral_constant<int, PM_BC_COLUMN>{});
}

// The unit stiffness in the form the kernel reads: the FP32 stencils on box
// cells take the 48 values by value (scalar registers, loaded once per wave);
// the FP64 stencils read the 576-entry table, since 48 doubles would take
// nearly all scalar registers and the compiler then spills them to vector
// lanes.
template <class T, class F>
void with_coeffs(const LatticeOp& op, F&& f) {
  if (op.cube) {
    KCube<T> K;
    memcpy(K.k, std::is_same<T, float>::value ? (const void*)op.kc32 : (const void*)op.kc64, sizeof(K.k));
    f(K);
    return;
  }
  if constexpr (std::is_same<T, float>::value) {
    if (op.sym) {
      KSym<float> K;
      memcpy(K.k, op.ks32, sizeof(K.k));
      f(K);
      return;
    }
  }
  f(KDense<T>{lat_K<T>(op)});
}

}  // namespace

template <class T>
void lattice_cheb_step(hipStream_t s, const Grid& G, const LatticeOp& op, const T* dinv, const T* b, const T* xin,
                       T* xout, T* d, T c1, T c2) {
  with_bc_kind(op.kind, [&](auto kd) {
    with_coeffs<T>(op, [&](auto K) {
      k_lat_cheb<T, decltype(kd)::value, decltype(K)><<<blocks_for(G.nn), kBlock, 0, s>>>(G, K, lat_E<T>(op), dinv, b,
                                                                                       xin, xout, d, c1, c2);
    });
  });
  PM_CHECK_LAUNCH();
}
template void lattice_cheb_step<double>(hipStream_t, const Grid&, const LatticeOp&, const double*, const double*,
                                        const double*, double*, double*, double, double);
template void lattice_cheb_step<float>(hipStream_t, const Grid&, const LatticeOp&, const float*, const float*,
                                       const float*, float*, float*, float, float);

template <class T>
void lattice_residual(hipStream_t s, const Grid& G, const LatticeOp& op, const T* b, const T* x, T* r) {
  with_bc_kind(op.kind, [&](auto kd) {
    with_coeffs<T>(op, [&](auto K) {
      k_lat_residual<T, decltype(kd)::value, decltype(K)><<<blocks_for(G.nn), kBlock, 0, s>>>(G, K, lat_E<T>(op), b,
                                                                                           x, r);
    });
  });
  PM_CHECK_LAUNCH();
}
template void lattice_residual<double>(hipStream_t, const Grid&, const LatticeOp&, const double*, const double*,
                                       double*);
template void lattice_residual<float>(hipStream_t, const Grid&, const LatticeOp&, const float*, const float*,
                                      float*);

template <class T>
void lattice_apply_t(hipStream_t s, const Grid& G, const LatticeOp& op, const T* x, T* y) {
  with_bc_kind(op.kind, [&](auto kd) {
    with_coeffs<T>(op, [&](auto K) {
      k_lat_apply<T, decltype(kd)::value, decltype(K)><<<blocks_for(G.nn), kBlock, 0, s>>>(G, K, lat_E<T>(op), x,
                                                                                           y);
    });
  });
  PM_CHECK_LAUNCH();
}
void lattice_apply(hipStream_t s, const Grid& G, const LatticeOp& op, const double* x, double* y) {
  lattice_apply_t<double>(s, G, op, x, y);
}
void lattice_apply(hipStream_t s, const Grid& G, const LatticeOp& op, const float* x, float* y) {
  lattice_apply_t<float>(s, G, op, x, y);
}

template <class TX>
void lattice_ah_u(hipStream_t s, const Grid& G, const LatticeOp& op, const TX* u, const TX* p, double sgn,
                  double* y) {
  with_bc_kind(op.kind, [&](auto kd) {
    with_coeffs<double>(op, [&](auto K) {
      k_lat_ah_u<TX, decltype(kd)::value, decltype(K)><<<blocks_for(G.nn), kBlock, 0, s>>>(G, K, op.ah, op.E, u, p,
                                                                                          sgn, y);
    });
  });
  PM_CHECK_LAUNCH();
}
template void lattice_ah_u<double>(hipStream_t, const Grid&, const LatticeOp&, const double*, const double*, double,
                                   double*);
template void lattice_ah_u<float>(hipStream_t, const Grid&, const LatticeOp&, const float*, const float*, double,
                                  double*);

void lattice_deviation(hipStream_t s, const Grid& G, const double* coords, double* dev, double* hmin) {
  unsigned long long* out = dalloc<unsigned long long>(1);
  PM_HIP(hipMemsetAsync(out, 0, sizeof(unsigned long long), s));
  k_lat_dev<<<blocks_for(G.nn), kBlock, 0, s>>>(G, coords, out);
  PM_CHECK_LAUNCH();
  unsigned long long bits = 0;
  double X[4][3];
  const int64_t ids[4] = {0, G.node(1, 0, 0), G.node(0, 1, 0), G.node(0, 0, 1)};
  PM_HIP(hipMemcpyAsync(&bits, out, sizeof(bits), hipMemcpyDeviceToHost, s));
  for (int q = 0; q < 4; ++q)
    PM_HIP(hipMemcpyAsync(X[q], coords + 3 * ids[q], 3 * sizeof(double), hipMemcpyDeviceToHost, s));
  PM_HIP(hipStreamSynchronize(s));
  dfree(out);
  double d;
  static_assert(sizeof(d) == sizeof(bits), "");
  memcpy(&d, &bits, sizeof(d));
  *dev = d;
  double h = 1e300;
  for (int q = 1; q < 4; ++q) {
    const double e0 = X[q][0] - X[0][0], e1 = X[q][1] - X[0][1], e2 = X[q][2] - X[0][2];
    h = std::min(h, std::sqrt(e0 * e0 + e1 * e1 + e2 * e2));
  }
  *hmin = h;
}

// After the unit element matrix is computed: whether the cell is a box (the
// 48 values rebuild every entry of Khat), and those values (synchronizes).
void lattice_unit(pm_ctx* c) {
  LatticeOp& op = c->lat;
  double K[576];
  PM_HIP(hipMemcpyAsync(K, op.Kh, sizeof(K), hipMemcpyDeviceToHost, c->s));
  PM_HIP(hipStreamSynchronize(c->s));
  double kmax = 0.0;
  for (double v : K) kmax = std::max(kmax, std::fabs(v));
  for (int d = 0; d < 8; ++d)
    for (int r = 0; r < 3; ++r)
      for (int q = r; q < 3; ++q) op.ks64[6 * d + sym_slot(r, q)] = K[r * 24 + 3 * d + q];
  bool sym = kmax > 0.0;
  for (int a = 0; a < 8 && sym; ++a)
    for (int b = 0; b < 8; ++b)
      for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) {
          const double v = op.ks64[6 * (a ^ b) + sym_slot(r, q)];
          const double want = sym_negated(a, b, r, q) ? -v : v;
          if (std::fabs(K[(3 * a + r) * 24 + 3 * b + q] - want) > 1e-13 * kmax) sym = false;
        }
  op.sym = sym;
  for (int i = 0; i < 48; ++i) op.ks32[i] = (float)op.ks64[i];
  // cubic cells: one value per slot, from the first entry that has it
  bool have[12] = {};
  for (int d = 0; d < 8; ++d)
    for (int r = 0; r < 3; ++r)
      for (int q = r; q < 3; ++q) {
        const int sl = cube_slot(d, r, q);
        if (!have[sl]) {
          const double v = K[r * 24 + 3 * d + q];
          op.kc64[sl] = cube_negated(d, r, q) ? -v : v;
          have[sl] = true;
        }
      }
  bool cube = sym;
  for (int a = 0; a < 8 && cube; ++a)
    for (int b = 0; b < 8; ++b)
      for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) {
          const int d = a ^ b, lo = r < q ? r : q, hi = r < q ? q : r;
          const double v = op.kc64[cube_slot(d, lo, hi)];
          const double want = (sym_negated(a, b, r, q) != cube_negated(d, lo, hi)) ? -v : v;
          if (std::fabs(K[(3 * a + r) * 24 + 3 * b + q] - want) > 1e-13 * kmax) cube = false;
        }
  op.cube = cube;
  for (int i = 0; i < 12; ++i) op.kc32[i] = (float)op.kc64[i];
}

// After assembly on a lattice: FP32 copies and the operator description.
void lattice_finish(pm_ctx* c) {
  LatticeOp& op = c->lat;
  op.kind = c->bc_kind;
  op.E = c->E;
  if (c->opts.precond_fp32) {
    if (!op.Kh32) op.Kh32 = dalloc<float>(576);
    if (!op.E32) op.E32 = dalloc<float>(c->nc);
    k_lat_to_float<<<blocks_for(576), kBlock, 0, c->s>>>(576, op.Kh, op.Kh32);
    k_lat_to_float<<<blocks_for(c->nc), kBlock, 0, c->s>>>(c->nc, c->E, op.E32);
    PM_CHECK_LAUNCH();
  }
  op.on = true;
}

}  // namespace pm
