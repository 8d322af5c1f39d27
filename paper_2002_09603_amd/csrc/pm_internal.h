// Internal declarations of the poromechanics step library (gfx950).
// Not part of the C ABI: see include/poromech.h for the public interface.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <functional>
#include <stdexcept>
#include <string>
#include <vector>

#include "poromech.h"
#include "pm_geom.h"

namespace pm {

// ---------------------------------------------------------------------------
// errors: internal code throws pm::Error; the C ABI layer converts it to a
// return code and keeps the message in the context.
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define PM_HIP(call)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      throw ::pm::Error(PM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_) +   \
                                     " (" + __FILE__ + ":" + std::to_string(__LINE__) + ")"); \
  } while (0)

#define PM_CHECK_LAUNCH() PM_HIP(hipGetLastError())

constexpr int kSlice = 64;   // SELL slice height = one wavefront of rows
constexpr int kSellWindow = 8;  // slices per window within which rows are sorted by length
constexpr int kBlock = 256;  // default threads per workgroup for streaming kernels

inline int blocks_for(int64_t n, int bs = kBlock) { return (int)((n + bs - 1) / bs); }

// ---------------------------------------------------------------------------
// kernel profiler: HIP events around the launches of selected kernels on
// their own stream, with the algorithmic bytes each launch must move
enum ProfKernel : int {
  kProfAHu = 1,          // u-rows of A_H (FP64, lattice or assembled A_uu, fused coupling)
  kProfChebU0 = 2,       // fused Chebyshev step on the finest A_uu level
  kProfChebPi0 = 3,      // fused Chebyshev step on the finest C~_pi level
  kProfMultidot = 4,     // FGMRES multi-dot (Gram-Schmidt projections)
  kProfMultiaxpy = 5,    // FGMRES Gram-Schmidt update (orthogonalise + normalise, or multi-AXPY)
  kProfRestrictU0 = 6,   // restriction from the finest A_uu level
  kProfAHp = 7,          // p-rows of A_H
  kProfAHpi = 8,         // pi-rows of A_H
  kProfProlongU0 = 9,    // prolongation onto the finest A_uu level
  kProfRestrictPi0 = 10, // restriction from the finest C~_pi level
  kProfProlongPi0 = 11,  // prolongation onto the finest C~_pi level
  kProfResidU0 = 12,     // residual on the finest A_uu level
  kProfResidPi0 = 13,    // residual on the finest C~_pi level
  kProfCount = 14
};

// Per launch: algorithmic bytes (stored values and indices, each input vector
// read once, each output written once) and, for the matrix-free lattice
// stencils, whose arithmetic bounds them, the multiply-add flops (2 per
// multiply-add of the stencil; 0 for memory-bound kernels).
struct Profiler {
  unsigned mask = 0;
  struct Rec {
    hipEvent_t a = nullptr, b = nullptr;
    double bytes = 0.0;
    double flops = 0.0;
  };
  std::vector<Rec> recs[kProfCount];
  size_t used[kProfCount] = {0};
  bool on(int k) const { return (mask >> k) & 1u; }
  void begin(hipStream_t s, int k);
  void end(hipStream_t s, int k, double bytes, double flops = 0.0);
  void reset(unsigned m);
  // sums over recorded launches of kernel k (synchronizes the events)
  void collect(int k, int64_t* n, double* ms, double* bytes, double* flops);
};
extern Profiler g_prof;

// ---------------------------------------------------------------------------
// device memory
void* dmalloc(size_t bytes);
void dfree(void* p);
void set_alloc_stream(hipStream_t s);   // stream whose free lists dmalloc/dfree use
void release_device_cache();            // hipFree every cached block
template <class T> T* dalloc(int64_t n) { return (T*)dmalloc(sizeof(T) * (size_t)(n > 0 ? n : 1)); }

// Block compressed sparse row, square blocks of size bs (1 or 3), row-major
// blocks, columns sorted ascending within a row.
struct Csr {
  int bs = 1;
  int n = 0, m = 0;       // block rows, block columns
  int64_t nnzb = 0;
  int* rowptr = nullptr;  // n+1
  int* col = nullptr;     // nnzb
  double* val = nullptr;  // nnzb*bs*bs
  float* val32 = nullptr; // optional FP32 copy of val
  bool borrowed = false;  // arrays owned elsewhere: free_all only forgets them
  void free_all();
};

// Sliced ELL with slices of 64 block rows.  Entry column c of a slice holds one
// block per row (lane): col[c*64 + lane], val[(c*bs*bs + e)*64 + lane].
// Padding slots have col = -1 and zero values.
struct Sell {
  int bs = 1;
  int n = 0, m = 0;
  int nslices = 0;
  int64_t ncols = 0;        // total entry columns over all slices
  int64_t nnzb = 0;         // stored blocks of the source matrix (no padding)
  int* sptr = nullptr;      // nslices+1 (entry-column offsets)
  int* perm = nullptr;      // 3x3 blocks: row held by each slot (rows sorted by length within
                            // windows of kSellWindow slices, -1 empty); null: slot t holds row t
  int* col = nullptr;       // ncols*64
  double* val = nullptr;    // ncols*64*bs*bs
  float* val32 = nullptr;   // FP32 copy (mixed precision) or null
  void free_all();
};

// One AMG level: operator, smoother data, transfers to the next level.
struct Level {
  int bs = 1, n = 0;
  Csr A;                     // kept for the Galerkin products
  Sell As;                   // operator used by the cycle (sliced ELL) ...
  bool csr_cycle = false;    // ... or A itself, csr_lanes lanes per row (coarse levels)
  int csr_lanes = 16;
  double* dinv = nullptr;    // n*bs*bs inverse diagonal blocks
  float* dinv32 = nullptr;
  Sell P;                    // prolongation from level+1 (empty on the coarsest level)
  Csr R;                     // restriction P^T (long rows: applied with 16 lanes per row)
  double lmax = 0.0;         // estimate of lambda_max(D^-1 A)
  // work vectors (n*bs each)
  double *x = nullptr, *b = nullptr, *r = nullptr, *d = nullptr, *t = nullptr;
  float *xf = nullptr, *bf = nullptr, *rf = nullptr, *df = nullptr, *tf = nullptr;
  void free_all();
};

struct AmgParams {
  double theta = 0.0;
  int coarse_max = 64;
  int max_levels = 12;
  int cheb_degree = 2;
  int cycles = 1;                  // V-cycles per application
  int agg_dist = 2;                // aggregation roots: distance-1 or distance-2 independent set
  double cheb_lower = 0.3;         // Chebyshev interval [lower*lmax, upper*lmax]
  double cheb_upper = 1.1;
  int power_its = 15;
  double p_trunc = 0.0;            // scalar prolongator truncation threshold (0: none)
  bool fp32 = false;
  hipStream_t side = nullptr;      // optional second stream for set-up power iterations
  bool rbm = false;                // rigid-body near kernel on the finest level (bs 3, structured)
  const double* coords = nullptr;  // node coordinates (n_n x 3, device) for it
};

// A_uu on a mesh whose cells are translates of one parallelepiped: every
// element stiffness is E_T times the unit-modulus matrix Khat of the first
// cell and every coupling column is ahat, so the finest level is applied from
// Khat, ahat and E without an assembled matrix.  Dirichlet rows and columns
// follow u_fixed (identity rows, zero columns).
// Mirror symmetry of a box cell: reflecting across the mid-plane normal to
// axis r maps corner a to a ^ (1 << r) and flips the r-th displacement
// component, so Khat[a][b](r,c) = s_r(a) s_c(a) Khat[0][a^b](r,c) with
// s_r(a) = -1 when bit r of a is set; with Khat symmetric, Khat[0][d](r,c) =
// s_r(d) s_c(d) Khat[0][d](c,r).  A table of 48 holds Khat[0][d](r,c) for
// r <= c at 6d + sym_slot(r,c), in the order (0,0) (1,1) (2,2) (0,1) (0,2)
// (1,2).
__host__ __device__ constexpr int sym_slot(int r, int c) {
  return r == c ? r : ((r < c ? r : c) == 0 ? 2 + (r < c ? c : r) : 5);
}
__host__ __device__ constexpr bool sym_negated(int a, int b, int r, int c) {
  const int d = a ^ b;
  const bool n = ((a >> r) ^ (a >> c)) & 1;
  return (r > c && (((d >> r) ^ (d >> c)) & 1)) ? !n : n;
}

// Cubic cells add the axis permutations: Khat[0][d](r,c) for r <= c takes 12
// values, by the number of axes in d and whether r and c are among them
// (cube_slot); where exactly one of r, c is among them the value changes sign
// with the order of the pair (positive when r, the smaller, is).
__host__ __device__ constexpr int cube_slot(int d, int r, int c) {
  return ((d & 1) + ((d >> 1) & 1) + ((d >> 2) & 1)) == 0   ? (r == c ? 0 : 1)
         : ((d & 1) + ((d >> 1) & 1) + ((d >> 2) & 1)) == 3 ? (r == c ? 10 : 11)
         : ((d & 1) + ((d >> 1) & 1) + ((d >> 2) & 1)) == 1
             ? (r == c ? (((d >> r) & 1) ? 2 : 3) : ((((d >> r) | (d >> c)) & 1) ? 4 : 5))
             : (r == c ? (((d >> r) & 1) ? 6 : 7) : ((((d >> r) & (d >> c)) & 1) ? 8 : 9));
}
__host__ __device__ constexpr bool cube_negated(int d, int r, int c) {
  return (cube_slot(d, r, c) == 4 || cube_slot(d, r, c) == 9) && !((d >> r) & 1);
}

struct LatticeOp {
  bool on = false;
  int kind = 0;               // boundary-condition kind
  double* Kh = nullptr;       // 576, row-major 24x24 (rows 3a+r, columns 3b+s)
  float* Kh32 = nullptr;
  double* ah = nullptr;       // 24 coupling column
  const double* E = nullptr;  // n_c moduli (context-owned)
  float* E32 = nullptr;       // FP32 copy for mixed precision
  // Box cells (mirror-symmetric in each axis): Khat is fixed by the 8 blocks
  // Khat[0][d], each symmetric up to signs, 48 values in all, passed to the
  // stencil kernels by value (kept in scalar registers)
  bool sym = false;
  double ks64[48] = {};
  float ks32[48] = {};
  bool cube = false;  // cubic cells: the 12 values kc64/kc32 rebuild Khat
  double kc64[12] = {};
  float kc32[12] = {};
  void free_all();
};

// Launchers of the lattice kernels (pm_lattice.hip); one thread per node.
// Chebyshev step: r = D^-1 (b - A x_in); d = c1 d + c2 r; x_out = x_in + d
template <class T>
void lattice_cheb_step(hipStream_t s, const Grid& G, const LatticeOp& op, const T* dinv, const T* b, const T* xin,
                       T* xout, T* d, T c1, T c2);
template <class T>
void lattice_residual(hipStream_t s, const Grid& G, const LatticeOp& op, const T* b, const T* x, T* r);
void lattice_apply(hipStream_t s, const Grid& G, const LatticeOp& op, const double* x, double* y);
void lattice_apply(hipStream_t s, const Grid& G, const LatticeOp& op, const float* x, float* y);  // E32, FP32 unit matrix
// u-rows of A_H: y_u = A_uu u + sgn A_up p (free rows), y_u = u (Dirichlet rows);
// FP64 arithmetic, FP64 or FP32 inputs
template <class TX>
void lattice_ah_u(hipStream_t s, const Grid& G, const LatticeOp& op, const TX* u, const TX* p, double sgn,
                  double* y);
// max over nodes of |X(i,j,k) - X(0) - i a - j b - k c| with a, b, c the edge
// vectors at node 0, and min |a|,|b|,|c| (synchronizes)
void lattice_deviation(hipStream_t s, const Grid& G, const double* coords, double* dev, double* hmin);

// C~_pi applied cell by cell from its element matrices (pm_cellpi.hip), FP64
// and an optional FP32 copy, structure of arrays [q*n_c + cell]:
//   full:  packed symmetric 6x6, q = pk(a,b) for a <= b (21 per cell);
//   block: M_T^-1 by direction blocks (q < 9, the layout of pm_ctx::Mb) and
//          q = 9: dt / B~_T, the element matrix being M^-1 - (dt/B~) g g^T
//          with g = M^-1 1 (10 per cell).
struct CellPiOp {
  bool on = false;
  bool block = false;
  int nvals = 0;  // values per cell of the allocated arrays
  double* C = nullptr;
  float* C32 = nullptr;
  void free_all();
};
template <class T>
void cellpi_cheb_step(hipStream_t s, const Grid& G, const CellPiOp& op, const T* dinv, const T* b, const T* xin,
                      T* xout, T* d, T c1, T c2);
template <class T>
void cellpi_residual(hipStream_t s, const Grid& G, const CellPiOp& op, const T* b, const T* x, T* r);
void cellpi_apply(hipStream_t s, const Grid& G, const CellPiOp& op, const double* x, double* y);
void cellpi_apply(hipStream_t s, const Grid& G, const CellPiOp& op, const float* x, float* y);  // C32

struct Hierarchy {
  int bs = 1;
  const LatticeOp* lat = nullptr;  // finest level applied on the lattice (A_uu only)
  const CellPiOp* cpi = nullptr;   // finest level applied cell by cell (C~_pi only)
  Grid grid{};                     // mesh of the lattice operator
  std::vector<Level> L;
  double* coarse_inv = nullptr;  // dense inverse of the coarsest operator (FP64)
  int ncoarse = 0;               // scalar size of the coarsest operator
  double* cwork = nullptr;       // 2*ncoarse scratch
  double *r0 = nullptr, *c0 = nullptr;   // finest-level residual/correction of iterated cycles
  float *r0f = nullptr, *c0f = nullptr;
  double opcx = 0.0;
  bool fp32 = false;
  AmgParams prm;
  void free_all();
};

}  // namespace pm

// ---------------------------------------------------------------------------
// the context (opaque in the C ABI)
struct pm_ctx {
  hipStream_t s = nullptr;
  hipStream_t s_aux = nullptr;  // library-owned second stream (C~_pi hierarchy set-up)
  hipStream_t s_side_u = nullptr, s_side_pi = nullptr;  // set-up power iterations of each hierarchy
  int nx = 0, ny = 0, nz = 0;
  int64_t nn = 0, nc = 0, nfx = 0, nfy = 0, nfz = 0, nf = 0, nmacro = 0;
  int64_t n_u = 0, n_p = 0, n_pi = 0, N = 0;
  double nu = 0.25, biot = 1.0, S = 0.0, mu = 1.0, dt = 1e-2;
  double trac[3] = {0, 0, -1};
  double p_top = 0.0;
  int bc_kind = PM_BC_COLUMN;
  pm_opts opts{};
  // inputs on the device
  double* coords = nullptr;  // nn*3
  double* E = nullptr;       // nc
  double* kappa = nullptr;   // nc*3
  // element data (structure-of-arrays, index [k*nc + cell])
  double* Ke = nullptr;      // 576*nc element stiffness (assembly scratch; unused on lattices)
  bool lattice = false;      // cells are translates of one parallelepiped
  pm::LatticeOp lat;         // finest-level A_uu operator on lattices
  pm::CellPiOp cpi;          // finest-level C~_pi operator from element matrices
  double* ae = nullptr;      // 24*nc coupling column of A_up
  double* vol = nullptr;     // nc
  double* Minv = nullptr;    // 36*nc inverse RT0 mass
  double* Mp = nullptr;      // 21*nc packed upper triangle of M^-1 (operator pi-rows)
  bool mblock = false;       // M^-1 couples only the two faces of each direction (beyond rounding)
  double* Mq = nullptr;      // 36*nc RT0 mass M_T, for the MFE operator (built on first use)
  bool Mq_valid = false;
  double* Mb = nullptr;      // 9*nc its blocks: [3d] (2d,2d), [3d+1] (2d,2d+1), [3d+2] (2d+1,2d+1)
  double* g = nullptr;       // 6*nc  M^-1 1
  double* alpha = nullptr;   // nc    1^T M^-1 1
  double* stabw = nullptr;   // nmacro: beta_M |M|
  double* bp = nullptr;      // nc: B~_p
  double* auu_diag = nullptr;// n_u scalar diagonal of A_uu
  uint8_t* ufix = nullptr;   // n_u
  uint8_t* pifix = nullptr;  // n_pi
  int* status = nullptr;     // device status word (inverted element, NaN, ...)
  // assembled operators
  pm::Csr Auu, Cpi, Cp;    // Cp: C~_p of the MFE preconditioner (built on first use)
  pm::Hierarchy Hu, Hpi, Hcp;  // Hcp: FP64 AMG hierarchy of the MFE C~_p
  // MFE block triangular preconditioner, built on first use and kept until
  // the next assembly or change of dt
  bool mfe_valid = false;
  bool auu_cols_set = false;  // A_uu column indices written (fixed pattern)
  double* mfe_lq = nullptr;    // n_pi absolute row sums of the masked A_qq (1 on no-flow faces)
  double* mfe_dqinv = nullptr; // n_pi inverse diagonal of the masked A_qq
  double mfe_qmax = 0.0;       // Gershgorin bound of lambda_max(D^-1 A_qq)
  double* mfe_work = nullptr;  // 3 n_pi + n_p + 256: A_qq sweep vectors, C~_p right-hand side, set-up maxima
  bool assembled = false;
  bool hier_u_ok = false;
  double fill_s = 0.0;       // kernel time of the last A_uu value fill (booked as assembly)
  // Krylov workspace
  int m_alloc = 0;
  int64_t ld = 0;            // distance between consecutive Krylov vectors (N rounded up to 32)
  double* V = nullptr;       // (m+1)*ld
  double* Z = nullptr;       // m*N preconditioned vectors (FP64 preconditioner, or two-pass Gram-Schmidt)
  float* Zf = nullptr;       // m*N preconditioned vectors from the FP32 preconditioner
  int mz_alloc = 0, mzf_alloc = 0;
  double* wvec = nullptr;    // N
  double* rvec = nullptr;    // N
  double* xvec = nullptr;    // N
  double* red = nullptr;     // reduction partials
  double* hcol = nullptr;    // device scalars (m+2)
  double* hhost = nullptr;   // pinned host copy
  // preconditioner work (FP64 and FP32)
  double* pw64 = nullptr;    // N
  float* pw32 = nullptr;     // 2*N
  pm_info info{};
  std::string err;
};

namespace pm {
// topology helpers (host side)
inline int64_t node_id(const pm_ctx* c, int i, int j, int k) {
  return i + (int64_t)(c->nx + 1) * (j + (int64_t)(c->ny + 1) * k);
}

// assembly (pm_assemble.hip)
Grid grid_of(const pm_ctx* c);
void assemble_all(pm_ctx* c);          // element kernels, masks, A_uu pattern and diagonal
void assemble_auu(pm_ctx* c);          // A_uu values, FP32 lattice data, packed M^-1 (after assemble_all)
void lattice_unit(pm_ctx* c);          // box-cell symmetry of Khat (pm_lattice.hip, synchronizes)
void lattice_finish(pm_ctx* c);        // lattice operator tables after assembly (pm_lattice.hip)
void cellpi_build(pm_ctx* c, hipStream_t s);          // packed C~_pi element matrices (pm_cellpi.hip)
void build_cpi(pm_ctx* c, hipStream_t s);  // B~p, assembled C~pi for the current dt (after assemble_all)
void build_rhs(pm_ctx* c, const double* u_prev, const double* p_prev, double* b);
int check_status(pm_ctx* c, const char* where);  // throws on error bits, returns the word

// operators (pm_ops.hip)
void apply_AH(pm_ctx* c, const double* x, double* y, bool transpose);
void apply_mfe(pm_ctx* c, const double* x, double* y);   // A_M of the MFE system, order [u; q; p]
void cell_data(pm_ctx* c, double* Mfull);
void build_cp(pm_ctx* c);                                 // C~_p of the MFE preconditioner into c->Cp
// MFE block triangular preconditioner of eq. prec (pm_mfe.hip): C~_p, its
// hierarchy (parameters prm) and the Jacobi data of A_qq; then z = M^-1 r
void mfe_prec_setup(pm_ctx* c, const AmgParams& prm);
// u-rows of A_H (and of A_M) in FP64: A_uu u + A_up p, Dirichlet rows identity (pm_ops.hip)
void apply_ah_u(pm_ctx* c, const double* u, const double* p, double* yu);
void apply_btp(pm_ctx* c, const double* r, double* z);
void build_rhs_mfe(pm_ctx* c, const double* u_prev, const double* p_prev, double* b);
constexpr int kQqChebDegree = 5;                          // Chebyshev-Jacobi sweeps of A_qq per application
void apply_AH32(pm_ctx* c, const float* x, double* y, bool transpose);    // FP32 input, FP64 arithmetic
void apply_Minv(pm_ctx* c, const double* r, double* z, bool transpose);
void apply_Minv32(pm_ctx* c, const float* r, float* z, bool transpose);   // FP32 hierarchies only
void apply_csr(pm_ctx* c, const Csr& A, const double* x, double* y);
void pack_minv(pm_ctx* c);             // c->Mp (or c->Mb when c->mblock) from c->Minv
void reconstruct_w(pm_ctx* c, const double* p, const double* pi, double* w);
void grad(pm_ctx* c, const double* lam, const double* x, const double* p_prev, double* dk,
          double* dE);
void rhs_adjoint(pm_ctx* c, const double* lam, double* cvec);

// sparse utilities (pm_sparse.hip)
void exclusive_scan(hipStream_t s, const int* in, int* out, int n, int* total_host);
void exclusive_scan64(hipStream_t s, const int64_t* in, int64_t* out, int64_t n, int64_t* total_host);
void csr_to_sell(hipStream_t s, const Csr& A, Sell& S, bool with_fp32);
void sell_spmv(hipStream_t s, const Sell& A, const double* x, double* y);
void sell_spmv32(hipStream_t s, const Sell& A, const float* x, float* y);
void csr_transpose(hipStream_t s, const Csr& A, Csr& T);
// C = A B; ptent_agg (optional): B is the tentative prolongator of that
// aggregation (identity block in column agg[j] of row j), numeric phase by sums
void spgemm(hipStream_t s, const Csr& A, const Csr& B, Csr& C, const int* ptent_agg = nullptr);
void block_diag_inverse(hipStream_t s, const Csr& A, double* dinv);

// AMG (pm_amg.hip)
// lat / cpi (may be null): apply the finest level of a block-3 / scalar
// hierarchy with the lattice / cell operator on grid G instead of an
// assembled sliced-ELL matrix
void amg_setup(hipStream_t s, const Csr& A, const AmgParams& prm, Hierarchy& H, const LatticeOp* lat = nullptr,
               const Grid* G = nullptr, const CellPiOp* cpi = nullptr);
void amg_vcycle(hipStream_t s, Hierarchy& H, const double* b, double* x);       // FP64
void amg_vcycle32(hipStream_t s, Hierarchy& H, const float* b, float* x);       // FP32 levels

// Krylov (pm_krylov.hip)
// Device workspace of one FGMRES run: basis V ((m_cap+1) vectors of stride
// ld), preconditioned vectors Z (FP64) or Zf (FP32), reduction partial sums,
// device scalars and a host copy of them.
struct KrylovWs {
  int m_cap = 0;
  int64_t ld = 0;
  double* V = nullptr;
  double* Z = nullptr;
  float* Zf = nullptr;
  double* red = nullptr;
  double* hcol = nullptr;
  double* hhost = nullptr;  // host, m_cap + 8 doubles
};
// Host arrays of the Givens process: H ((m_cap+1) x m_cap), cs, sn, y (m_cap), g (m_cap+1)
struct KrylovHost {
  int m_cap = 0;
  double *H = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr, *y = nullptr;
};
// Operator and right preconditioner of the iteration (vectors of length c->N);
// the FP32 pair is used with one Gram-Schmidt pass when M32 is set.
struct KrylovOps {
  std::function<void(const double*, double*)> A64, M64;
  std::function<void(const float*, double*)> A32;
  std::function<void(const float*, float*)> M32;
};
int64_t krylov_ld(int64_t N);
void krylov_preload(hipStream_t s);                                // load the Krylov kernels' code object
size_t krylov_device_bytes(int64_t N, int m, bool z32);           // device bytes of krylov_ws_in
KrylovWs krylov_ws_in(void* base, size_t bytes, int64_t N, int m, bool z32);  // carve from a buffer
KrylovOps step_ops(pm_ctx* c, bool transpose);                     // A_H and M^-1 (or transposes)
int fgmres_ws(pm_ctx* c, const KrylovOps& op, const KrylovWs& ws, KrylovHost& hw, const double* b, double* x,
              pm_info* info);
int fgmres(pm_ctx* c, const double* b, double* x, bool transpose, pm_info* info);  // context workspace
int fgmres_with(pm_ctx* c, const KrylovOps& op, const double* b, double* x, pm_info* info);  // same, any operator
}  // namespace pm

namespace pm {
// Row accumulation acc += sum over entry columns [e0, e1) of one SELL slice
// (lane = row within the slice).  Entry columns are taken in groups of U: the
// column ids, then the matrix blocks and the gathered x blocks of the whole
// group are loaded before any use, so each group costs two dependent memory
// latencies instead of two per entry.  The summation order is the entry order.
template <int BS, int U, class T, class TA>
__device__ inline void sell_row(int e0, int e1, const int* __restrict__ col, const T* __restrict__ val,
                                const T* __restrict__ x, int lane, TA acc[BS]) {
  int c = e0;
  for (; c + U <= e1; c += U) {
    int j[U];
#pragma unroll
    for (int u = 0; u < U; ++u) j[u] = col[(size_t)(c + u) * kSlice + lane];
    T v[U][BS * BS];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int q = 0; q < BS * BS; ++q)
        v[u][q] = __builtin_nontemporal_load(val + ((size_t)(c + u) * BS * BS + q) * kSlice + lane);
    T xj[U][BS];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int q = 0; q < BS; ++q) xj[u][q] = x[(size_t)j[u] * BS + q];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int a = 0; a < BS; ++a)
#pragma unroll
        for (int q = 0; q < BS; ++q) acc[a] += (TA)v[u][a * BS + q] * (TA)xj[u][q];
  }
  for (; c < e1; ++c) {
    const int jj = col[(size_t)c * kSlice + lane];
    T xj[BS];
#pragma unroll
    for (int q = 0; q < BS; ++q) xj[q] = x[(size_t)jj * BS + q];
#pragma unroll
    for (int a = 0; a < BS; ++a)
#pragma unroll
      for (int q = 0; q < BS; ++q)
        acc[a] += (TA)val[((size_t)c * BS * BS + a * BS + q) * kSlice + lane] * (TA)xj[q];
  }
}

// row held by SELL slot t (perm null: slot t holds row t), -1 for an empty slot
__device__ __forceinline__ int sell_row_of(const int* __restrict__ perm, int t, int n) {
  return perm ? perm[t] : (t < n ? t : -1);
}

template <int BS>
struct SellUnroll {
  static constexpr int value = BS == 3 ? 3 : 4;
};
}  // namespace pm
