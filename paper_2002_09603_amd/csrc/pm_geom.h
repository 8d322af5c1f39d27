// Device helpers for the structured hexahedral mesh and the trilinear map.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "poromech.h"

namespace pm {

// Division by a run-time constant d for 0 <= n < 2^31: q = (n m) >> sh with
// L = ceil(log2 d), sh = 31 + L, m = ceil(2^sh / d) < 2^32 (Granlund and
// Montgomery, "Division by invariant integers using multiplication", 1994).
struct FastDiv {
  uint32_t d = 1, m = 0x80000000u;
  int sh = 31;
  __host__ void init(uint32_t dd) {
    d = dd;
    int L = 0;
    while ((1ull << L) < dd) ++L;
    sh = 31 + L;
    m = (uint32_t)(((1ull << sh) + dd - 1) / dd);
  }
  __host__ __device__ uint32_t div(uint32_t n) const { return (uint32_t)(((uint64_t)n * m) >> sh); }
};

// Structured grid description passed by value to kernels.  Index arithmetic
// assumes fewer than 2^31 nodes, cells and faces (checked at set-up).
struct Grid {
  int nx, ny, nz;
  int drained;  // 1: the top plane's faces are Dirichlet (drained); 0: no-flow everywhere
  int64_t nn, nc, nfx, nfy, nfz, nf;
  FastDiv dnx, dnx1, dny, dny1;  // division by nx, nx+1, ny, ny+1
  __host__ __device__ int64_t node(int i, int j, int k) const {
    return i + (int64_t)(nx + 1) * (j + (int64_t)(ny + 1) * k);
  }
  __host__ __device__ int64_t cell(int i, int j, int k) const {
    return i + (int64_t)nx * (j + (int64_t)ny * k);
  }
  __host__ __device__ int64_t fx(int i, int j, int k) const {
    return i + (int64_t)(nx + 1) * (j + (int64_t)ny * k);
  }
  __host__ __device__ int64_t fy(int i, int j, int k) const {
    return nfx + i + (int64_t)nx * (j + (int64_t)(ny + 1) * k);
  }
  __host__ __device__ int64_t fz(int i, int j, int k) const {
    return nfx + nfy + i + (int64_t)nx * (j + (int64_t)ny * k);
  }
  __host__ __device__ int64_t macro(int ci, int cj, int ck) const {
    return (ci >> 1) + (int64_t)(nx >> 1) * ((cj >> 1) + (int64_t)(ny >> 1) * (ck >> 1));
  }
  // local faces (-x,+x,-y,+y,-z,+z) of cell (i,j,k)
  __host__ __device__ void cell_faces(int i, int j, int k, int64_t f[6]) const {
    f[0] = fx(i, j, k);
    f[1] = fx(i + 1, j, k);
    f[2] = fy(i, j, k);
    f[3] = fy(i, j + 1, k);
    f[4] = fz(i, j, k);
    f[5] = fz(i, j, k + 1);
  }
  __host__ __device__ void cell_ijk(int64_t c, int& i, int& j, int& k) const {
    const uint32_t u = (uint32_t)c, r = dnx.div(u), kk = dny.div(r);
    i = (int)(u - r * (uint32_t)nx);
    j = (int)(r - kk * (uint32_t)ny);
    k = (int)kk;
  }
  __host__ __device__ void node_ijk(int64_t n, int& i, int& j, int& k) const {
    const uint32_t u = (uint32_t)n, r = dnx1.div(u), kk = dny1.div(r);
    i = (int)(u - r * (uint32_t)(nx + 1));
    j = (int)(r - kk * (uint32_t)(ny + 1));
    k = (int)kk;
  }
  // cells adjacent to face f: cell ids (or -1) and the local face index in each
  __host__ __device__ void face_cells(int64_t f, int64_t c[2], int lf[2]) const {
    int i, j, k;
    if (f < nfx) {
      const uint32_t u = (uint32_t)f, r = dnx1.div(u), kk = dny.div(r);
      i = (int)(u - r * (uint32_t)(nx + 1));
      j = (int)(r - kk * (uint32_t)ny);
      k = (int)kk;
      c[0] = i > 0 ? cell(i - 1, j, k) : -1;
      lf[0] = 1;
      c[1] = i < nx ? cell(i, j, k) : -1;
      lf[1] = 0;
    } else if (f < nfx + nfy) {
      const uint32_t u = (uint32_t)(f - nfx), r = dnx.div(u), kk = dny1.div(r);
      i = (int)(u - r * (uint32_t)nx);
      j = (int)(r - kk * (uint32_t)(ny + 1));
      k = (int)kk;
      c[0] = j > 0 ? cell(i, j - 1, k) : -1;
      lf[0] = 3;
      c[1] = j < ny ? cell(i, j, k) : -1;
      lf[1] = 2;
    } else {
      const uint32_t u = (uint32_t)(f - nfx - nfy), r = dnx.div(u), kk = dny.div(r);
      i = (int)(u - r * (uint32_t)nx);
      j = (int)(r - kk * (uint32_t)ny);
      k = (int)kk;
      c[0] = k > 0 ? cell(i, j, k - 1) : -1;
      lf[0] = 5;
      c[1] = k < nz ? cell(i, j, k) : -1;
      lf[1] = 4;
    }
  }
};

// Dirichlet displacement components of node (i,j,k): the bottom face is
// fixed; PM_BC_ROLLERS also fixes the normal component on the lateral faces;
// PM_BC_CANTILEVER fixes the face x = x_min instead.
__host__ __device__ inline bool u_fixed(const Grid& G, int kind, int i, int j, int k, int comp) {
  if (kind == PM_BC_CANTILEVER) return i == 0;
  if (k == 0) return true;
  if (kind != PM_BC_ROLLERS) return false;
  if (comp == 0) return i == 0 || i == G.nx;
  if (comp == 1) return j == 0 || j == G.ny;
  return false;
}

// Dirichlet face pressures: the faces of the top plane when it is drained.
__host__ __device__ inline bool pi_fixed(const Grid& G, int64_t f) {
  return G.drained && f >= G.nf - (int64_t)G.nx * G.ny;  // z-faces numbered last, plane k = nz at the end
}
// the same for local face e of cell (., ., k): only the +z face of a top cell
__host__ __device__ inline bool pi_fixed_local(const Grid& G, int k, int e) {
  return G.drained && e == 5 && k == G.nz - 1;
}

// packed index of (a, b), a <= b, in the row-major upper triangle of a
// symmetric 6x6 matrix (21 entries)
__host__ __device__ inline int sym6(int a, int b) { return a * 6 - (a * (a - 1)) / 2 + (b - a); }

// base[idx] through a 32-bit byte offset from a (typically wave-uniform)
// base; valid for arrays of fewer than 2^32 bytes, which the set-up size
// limits guarantee for every per-node, per-cell and per-face array.
template <class T>
__device__ __forceinline__ T ld32(const T* __restrict__ base, uint32_t idx) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + idx * (uint32_t)sizeof(T));
}

// Faces of cell (ci,cj,ck) in 32-bit arithmetic, local order (-x,+x,-y,+y,-z,+z).
__device__ __forceinline__ void cell_faces32(const Grid& G, uint32_t ci, uint32_t cj, uint32_t ck, uint32_t F[6]) {
  const uint32_t nx = (uint32_t)G.nx, ny = (uint32_t)G.ny;
  F[0] = ci + (nx + 1) * (cj + ny * ck);
  F[1] = F[0] + 1;
  F[2] = (uint32_t)G.nfx + ci + nx * (cj + (ny + 1) * ck);
  F[3] = F[2] + nx;
  F[4] = (uint32_t)(G.nfx + G.nfy) + ci + nx * (cj + ny * ck);
  F[5] = F[4] + nx * ny;
}

// Position (i,j,k) of face f within its orientation (0: x, 1: y, 2: z).
__device__ __forceinline__ int face_pos(const Grid& G, uint32_t f, uint32_t& i, uint32_t& j, uint32_t& k) {
  const uint32_t nx = (uint32_t)G.nx, ny = (uint32_t)G.ny;
  if (f < (uint32_t)G.nfx) {
    const uint32_t r = G.dnx1.div(f);
    i = f - r * (nx + 1);
    k = G.dny.div(r);
    j = r - k * ny;
    return 0;
  }
  if (f < (uint32_t)(G.nfx + G.nfy)) {
    const uint32_t u = f - (uint32_t)G.nfx, r = G.dnx.div(u);
    i = u - r * nx;
    k = G.dny1.div(r);
    j = r - k * (ny + 1);
    return 1;
  }
  const uint32_t u = f - (uint32_t)(G.nfx + G.nfy), r = G.dnx.div(u);
  i = u - r * nx;
  k = G.dny.div(r);
  j = r - k * ny;
  return 2;
}

template <int L>
using LocalFace = std::integral_constant<int, L>;

// Calls fn(LocalFace<l>{}, c, F, ck) for each cell c adjacent to the face at
// (i,j,k) of orientation O, where l is the face's local index in c (a
// compile-time constant), F the six faces of c and ck its layer.
template <int O, class Fn>
__device__ __forceinline__ void visit_face_cells(const Grid& G, uint32_t i, uint32_t j, uint32_t k, Fn&& fn) {
  const uint32_t pos = O == 0 ? i : (O == 1 ? j : k);
  const uint32_t lim = (uint32_t)(O == 0 ? G.nx : (O == 1 ? G.ny : G.nz));
  const uint32_t nx = (uint32_t)G.nx, ny = (uint32_t)G.ny;
  if (pos > 0) {
    const uint32_t ci = i - (O == 0), cj = j - (O == 1), ck = k - (O == 2);
    uint32_t F[6];
    cell_faces32(G, ci, cj, ck, F);
    fn(LocalFace<2 * O + 1>{}, ci + nx * (cj + ny * ck), F, ck);
  }
  if (pos < lim) {
    uint32_t F[6];
    cell_faces32(G, i, j, k, F);
    fn(LocalFace<2 * O>{}, i + nx * (j + ny * k), F, k);
  }
}

// Face rows by owning cell: cell (i,j,k) owns its -x, -y and -z faces, and
// also its +x, +y, +z faces on the last layer of each direction, so every
// face has one owner.  For each owned face f, out(f, fixed, acc) receives the
// sum over the (one or two) cells T adjacent to f of
// term(LocalFace<l>{}, c_T, F_T, k_T), l the local index of f in T, F_T the
// six faces of T and k_T its layer; fixed marks the Dirichlet faces (a drained top
// plane), whose acc is not formed.  A thread per cell reads each cell's data
// for its own faces and its -x/-y/-z neighbours' data for the shared faces
// (neighbouring threads, so mostly from cache): the per-cell arrays cross HBM
// about once, where a thread per face re-reads them once per orientation.
template <int D, class T, class Term, class Out>
__device__ __forceinline__ void owned_face_dir(const Grid& G, uint32_t i, uint32_t j, uint32_t k, uint32_t c,
                                               const uint32_t F[6], Term& term, Out& out) {
  const uint32_t nx = (uint32_t)G.nx, ny = (uint32_t)G.ny;
  const uint32_t pos = D == 0 ? i : (D == 1 ? j : k);
  const uint32_t lim = (uint32_t)(D == 0 ? G.nx : (D == 1 ? G.ny : G.nz));
  // face F[2D]: this cell (local 2D) and the cell before it (local 2D+1)
  T acc = term(LocalFace<2 * D>{}, c, F, k);
  if (pos > 0) {
    const uint32_t bi = i - (D == 0), bj = j - (D == 1), bk = k - (D == 2);
    uint32_t Fb[6];
    cell_faces32(G, bi, bj, bk, Fb);
    acc += term(LocalFace<2 * D + 1>{}, bi + nx * (bj + ny * bk), Fb, bk);
  }
  out(F[2 * D], false, acc);
  // face F[2D+1] on the last layer: this cell only; a drained top plane is Dirichlet
  if (pos == lim - 1) {
    if (D == 2 && G.drained)
      out(F[5], true, (T)0);
    else
      out(F[2 * D + 1], false, term(LocalFace<2 * D + 1>{}, c, F, k));
  }
}

template <class T, class Term, class Out>
__device__ __forceinline__ void owned_face_rows(const Grid& G, uint32_t i, uint32_t j, uint32_t k, Term&& term,
                                                Out&& out) {
  const uint32_t c = i + (uint32_t)G.nx * (j + (uint32_t)G.ny * k);
  uint32_t F[6];
  cell_faces32(G, i, j, k, F);
  owned_face_dir<0, T>(G, i, j, k, c, F, term, out);
  owned_face_dir<1, T>(G, i, j, k, c, F, term, out);
  owned_face_dir<2, T>(G, i, j, k, c, F, term, out);
}

// Workgroups are dispatched to the 8 XCDs round-robin; this maps workgroup b
// of nb so that each XCD runs one contiguous range of logical workgroups
// (neighbour rows and planes gathered by a workgroup then sit in the L2 of
// the same XCD).
__device__ inline int64_t xcd_block(int64_t b, int64_t nb) {
  const int64_t q = nb / 8, r = nb % 8;
  const int64_t id = b % 8, idx = b / 8;
  return id < r ? id * (q + 1) + idx : r * (q + 1) + (id - r) * q + idx;
}

constexpr double kGauss = 0.57735026918962576451;  // 1/sqrt(3)

__host__ __device__ inline void gauss_point(int q, double xi[3]) {
  xi[0] = (q & 1) ? kGauss : -kGauss;
  xi[1] = ((q >> 1) & 1) ? kGauss : -kGauss;
  xi[2] = ((q >> 2) & 1) ? kGauss : -kGauss;
}

// reference gradient of the trilinear shape function of local node a
__host__ __device__ inline void ref_grad(int a, const double xi[3], double g[3]) {
  const double sx = (a & 1) ? 1.0 : -1.0;
  const double sy = ((a >> 1) & 1) ? 1.0 : -1.0;
  const double sz = ((a >> 2) & 1) ? 1.0 : -1.0;
  const double tx = 1.0 + sx * xi[0], ty = 1.0 + sy * xi[1], tz = 1.0 + sz * xi[2];
  g[0] = 0.125 * sx * ty * tz;
  g[1] = 0.125 * sy * tx * tz;
  g[2] = 0.125 * sz * tx * ty;
}

// J[i][j] = d x_i / d xi_j; returns det J
__host__ __device__ inline double jacobian(const double X[8][3], const double xi[3], double J[3][3]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) J[i][j] = 0.0;
  for (int a = 0; a < 8; ++a) {
    double g[3];
    ref_grad(a, xi, g);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) J[i][j] += X[a][i] * g[j];
  }
  return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
         J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
         J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

// inverse of J (given det)
__host__ __device__ inline void inv3(const double J[3][3], double det, double Ji[3][3]) {
  const double r = 1.0 / det;
  Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) * r;
  Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * r;
  Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * r;
  Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) * r;
  Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * r;
  Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * r;
  Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) * r;
  Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * r;
  Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * r;
}

// load the 8 node coordinates of cell (i,j,k)
__device__ inline void load_cell_coords(const Grid& G, const double* __restrict__ coords, int i, int j,
                                        int k, double X[8][3]) {
  for (int a = 0; a < 8; ++a) {
    const int64_t n = G.node(i + (a & 1), j + ((a >> 1) & 1), k + ((a >> 2) & 1));
    X[a][0] = coords[3 * n + 0];
    X[a][1] = coords[3 * n + 1];
    X[a][2] = coords[3 * n + 2];
  }
}

// status word bits written by kernels (read back by the host)
enum : int { kStatusInverted = 1, kStatusNonFinite = 2, kStatusCapacity = 4, kStatusBadPivot = 8 };
// informational bit (not an error): some cell's M_T^-1 couples faces of
// different directions beyond rounding
enum : int { kStatusFullMinv = 16 };

}  // namespace pm
