// Smoothed-aggregation AMG for the two SPD inner blocks of the block
// triangular preconditioner: A_uu (3x3 node blocks, translations per
// displacement component as near kernel: the "separate displacement
// component" variant) and C~_pi (scalar).  The paper uses PETSc GAMG and
// hypre BoomerAMG (Sec. 5); this is the project's own GPU design:
//
//  setup per level: symmetric strength of connection on block norms ->
//  distance-2 maximal independent set (Luby-type rounds on packed
//  (state, hash, id) tuples) -> aggregates = roots + distance-1 + distance-2
//  attachment -> tentative P (identity block per node) -> Jacobi-smoothed
//  P = (I - 4/(3 lmax) D^-1 A) P_tent -> Galerkin A_c = P^T (A P) by SpGEMM;
//  coarsest level inverted densely (Gauss-Jordan, FP64).
//
//  cycle: V(k,k) with Chebyshev(D^-1 A) smoothing (same polynomial before and
//  after, so the cycle is a symmetric operator and serves M^T as well).
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdlib>

#include "pm_internal.h"

namespace pm {

void Level::free_all() {
  A.free_all();
  As.free_all();
  P.free_all();
  R.free_all();
  dfree(dinv);
  dfree(dinv32);
  dfree(x);
  dfree(b);
  dfree(r);
  dfree(d);
  dfree(t);
  dfree(xf);
  dfree(bf);
  dfree(rf);
  dfree(df);
  dfree(tf);
  dinv = nullptr;
  dinv32 = nullptr;
  x = b = r = d = t = nullptr;
  xf = bf = rf = df = tf = nullptr;
}

void Hierarchy::free_all() {
  for (auto& l : L) l.free_all();
  L.clear();
  dfree(coarse_inv);
  dfree(cwork);
  dfree(r0);
  dfree(c0);
  dfree(r0f);
  dfree(c0f);
  coarse_inv = nullptr;
  cwork = nullptr;
  r0 = c0 = nullptr;
  r0f = c0f = nullptr;
  ncoarse = 0;
}

namespace {

enum : uint8_t { kUnd = 1, kIn = 2, kOut = 0 };

__device__ inline uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352dU;
  x ^= x >> 15;
  x *= 0x846ca68bU;
  x ^= x >> 16;
  return x;
}

template <int BS>
__device__ inline double block_norm(const double* v) {
  double s = 0.0;
  for (int q = 0; q < BS * BS; ++q) s += v[q] * v[q];
  return sqrt(s);
}

// Norms of the stored blocks for strength and aggregation.  3x3 blocks:
// computed once per entry into an array (one thread per block, coalesced),
// since three passes over the rows need them; scalars: |a| on the fly.
template <int BS>
struct BlockNorms {
  const double* p;  // BS == 3: per-entry norms; BS == 1: the values
  __device__ double operator()(int64_t e) const {
    if constexpr (BS == 1)
      return block_norm<1>(p + e);
    else
      return p[e];
  }
};

template <int BS>
__global__ void k_block_norms(int64_t nnzb, const double* __restrict__ val, double* __restrict__ nrm) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nnzb) nrm[e] = block_norm<BS>(val + (size_t)e * BS * BS);
}

// strength: strong[e] = 1 for off-diagonal |A_ij| >= theta sqrt(|A_ii||A_jj|), |A_ij| > 0;
// kZeroBlock for a stored block that is exactly zero (weak, but dropping it
// does not change the operator); 0 for the other weak couplings
constexpr uint8_t kZeroBlock = 2;
// The row kernels of strength and aggregation run G lanes per row (entries
// strided over the lanes, contiguous loads) and combine the lanes with
// shuffles; the results equal those of a sequential pass over each row.
template <int BS, int G>
__global__ void __launch_bounds__(256) k_diag_norm(int n, const int* __restrict__ rp, const int* __restrict__ col,
                                                   BlockNorms<BS> nv, double* __restrict__ dn) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = (int)(t / G), l = (int)(t % G);
  double v = 0.0;
  if (i < n)
    for (int e = rp[i] + l; e < rp[i + 1]; e += G)
      if (col[e] == i) v = nv(e);
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, G));  // one lane holds the (>= 0) norm
  if (i < n && l == 0) dn[i] = v;
}

template <int BS, int G>
__global__ void __launch_bounds__(256) k_strength(int n, const int* __restrict__ rp, const int* __restrict__ col,
                                                  BlockNorms<BS> nv, const double* __restrict__ dn, double theta,
                                                  uint8_t* __restrict__ strong, uint8_t* __restrict__ state) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = (int)(t / G), l = (int)(t % G);
  int ns = 0;
  if (i < n) {
    const double di = dn[i];
    for (int e = rp[i] + l; e < rp[i + 1]; e += G) {
      const int j = col[e];
      uint8_t sv = 0;
      if (j != i) {
        const double a = nv(e);
        sv = a == 0.0 ? kZeroBlock : (a >= theta * sqrt(di * dn[j]) ? 1 : 0);
      }
      strong[e] = sv;
      ns += sv == 1;
    }
  }
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) ns += __shfl_xor(ns, o, G);
  if (i < n && l == 0) state[i] = ns > 0 ? kUnd : kOut;  // isolated rows (e.g. Dirichlet) are never aggregated
}

// lanes' (best value, entry, target): the largest value, the first entry among ties
template <int G>
__device__ inline void argmax_lanes(double& best, int& eb, int& a) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) {
    const double ob = __shfl_xor(best, o, G);
    const int oe = __shfl_xor(eb, o, G), oa = __shfl_xor(a, o, G);
    if (ob > best || (ob == best && oe < eb)) {
      best = ob;
      eb = oe;
      a = oa;
    }
  }
}

// lanes per row for the row kernels: as for the independent-set passes
template <class F>
void with_row_lanes(const Csr& A, F&& f) {
  const double avg = (double)A.nnzb / std::max(1, A.n);
  if (avg <= 12.0)
    f(std::integral_constant<int, 4>{});
  else if (avg <= 40.0)
    f(std::integral_constant<int, 8>{});
  else
    f(std::integral_constant<int, 16>{});
}

__device__ inline uint64_t pack_tuple(uint8_t st, int i, uint32_t salt) {
  const uint64_t rank = st == kIn ? 2 : (st == kUnd ? 1 : 0);
  const uint64_t pr = mix32((uint32_t)i * 2654435761u + salt) & 0x3FFFFFFFu;
  return (rank << 62) | (pr << 32) | (uint32_t)i;
}

// The round kernels take go: a round whose predecessor left no undecided row
// is skipped on the device (*go == 0), so the host checks only every few rounds.
__global__ void k_mis_init(int n, const uint8_t* __restrict__ state, uint32_t salt, uint64_t* __restrict__ T0,
                           const int* __restrict__ go) {
  if (!*go) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) T0[i] = pack_tuple(state[i], i, salt);
}

// Tout[i] = max of Tin over i and its strong neighbours; G lanes per row
// stride over its entries (contiguous loads), then reduce with shuffles
template <int G>
__global__ void __launch_bounds__(256) k_mis_max(int n, const int* __restrict__ rp, const int* __restrict__ col,
                                                 const uint8_t* __restrict__ strong,
                                                 const uint64_t* __restrict__ Tin, uint64_t* __restrict__ Tout,
                                                 const int* __restrict__ go) {
  if (!*go) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = (int)(t / G), l = (int)(t % G);
  uint64_t m = 0;
  if (i < n) {
    if (l == 0) m = Tin[i];
    const int e1 = rp[i + 1];
    int e = rp[i] + l;
    // two entries per lane and step, loaded before either is compared
    for (; e + G < e1; e += 2 * G) {
      const bool s0 = strong[e] == 1, s1 = strong[e + G] == 1;
      const int c0 = col[e], c1 = col[e + G];
      const uint64_t v0 = s0 ? Tin[c0] : 0, v1 = s1 ? Tin[c1] : 0;
      m = v0 > m ? v0 : m;
      m = v1 > m ? v1 : m;
    }
    if (e < e1 && strong[e] == 1) {
      const uint64_t v = Tin[col[e]];
      m = v > m ? v : m;
    }
  }
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) {
    const uint32_t lo = __shfl_xor((uint32_t)m, o, G), hi = __shfl_xor((uint32_t)(m >> 32), o, G);
    const uint64_t v = ((uint64_t)hi << 32) | lo;
    m = v > m ? v : m;
  }
  if (i < n && l == 0) Tout[i] = m;
}

void launch_mis_max(hipStream_t s, const Csr& A, const uint8_t* strong, const uint64_t* Tin, uint64_t* Tout,
                    const int* go) {
  const double avg = (double)A.nnzb / std::max(1, A.n);
  if (avg <= 12.0)
    k_mis_max<4><<<blocks_for((int64_t)A.n * 4), kBlock, 0, s>>>(A.n, A.rowptr, A.col, strong, Tin, Tout, go);
  else if (avg <= 40.0)
    k_mis_max<8><<<blocks_for((int64_t)A.n * 8), kBlock, 0, s>>>(A.n, A.rowptr, A.col, strong, Tin, Tout, go);
  else
    k_mis_max<16><<<blocks_for((int64_t)A.n * 16), kBlock, 0, s>>>(A.n, A.rowptr, A.col, strong, Tin, Tout, go);
  PM_CHECK_LAUNCH();
}

// Finest levels on the structured mesh: the strong neighbours of a row as a
// bit mask over its stencil slots, so that each independent-set pass reads 4
// bytes per row (plus the neighbours' tuples, mostly from cache) instead of
// the CSR columns and strength flags.  The strong graph, and so the result
// of the rounds, is the same as on the CSR.
//   A_uu (node graph): slot (dk+1)*9 + (dj+1)*3 + (di+1) of neighbour (di,dj,dk).
//   C~_pi (face graph): slot 6*s + e = local face e of the cell on side s of
//   the face (s = 0: the cell below/left of it, 1: above/right).
// 32 lanes per row (a node has at most 27 blocks), OR-reduced with shuffles
__global__ void __launch_bounds__(256) k_mask_nodes(Grid G, const int* __restrict__ rp,
                                                    const int* __restrict__ col,
                                                    const uint8_t* __restrict__ strong, uint32_t* __restrict__ mask,
                                                    int* __restrict__ bad) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = t >> 5;
  const int l = (int)(t & 31);
  uint32_t m = 0;
  if (n < G.nn) {
    int i, j, k;
    G.node_ijk(n, i, j, k);
    const int sy = G.nx + 1, sz = sy * (G.ny + 1);
    for (int e = rp[n] + l; e < rp[n + 1]; e += 32) {
      if (strong[e] != 1) continue;
      // offset col - n = di + dj*sy + dk*sz with |di|, |dj|, |dk| <= 1, checked below
      const int d = col[e] - (int)n;
      const int dk = d > sz / 2 ? 1 : (d < -(sz / 2) ? -1 : 0);
      const int r = d - dk * sz;
      const int dj = r > sy / 2 ? 1 : (r < -(sy / 2) ? -1 : 0);
      const int di = r - dj * sy;
      const bool ok = di >= -1 && di <= 1 && i + di >= 0 && i + di <= G.nx && j + dj >= 0 && j + dj <= G.ny &&
                      k + dk >= 0 && k + dk <= G.nz;
      if (!ok) {
        *bad = 1;
        continue;
      }
      m |= 1u << ((dk + 1) * 9 + (dj + 1) * 3 + (di + 1));
    }
  }
#pragma unroll
  for (int o = 16; o > 0; o >>= 1) m |= __shfl_xor(m, o, 32);
  if (n < G.nn && l == 0) mask[n] = m;
}

__global__ void __launch_bounds__(256) k_mis_max_nodes(Grid G, const uint32_t* __restrict__ mask,
                                                       const uint64_t* __restrict__ Tin,
                                                       uint64_t* __restrict__ Tout, const int* __restrict__ go) {
  if (!*go) return;
  const int64_t n64 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n64 >= G.nn) return;
  const uint32_t n = (uint32_t)n64;
  const int sy = G.nx + 1, sz = (G.nx + 1) * (G.ny + 1);
  const uint32_t bits = mask[n];
  uint64_t m = Tin[n];
#pragma unroll
  for (int b = 0; b < 27; ++b) {
    if (b == 13 || !((bits >> b) & 1u)) continue;
    const int off = (b % 3 - 1) + (b / 3 % 3 - 1) * sy + (b / 9 - 1) * sz;
    const uint64_t v = ld32(Tin, (uint32_t)((int)n + off));
    m = v > m ? v : m;
  }
  Tout[n] = m;
}

// the (up to 12) faces of the two cells on either side of face f; absent
// cells give UINT32_MAX
__device__ inline void face_slots(const Grid& G, uint32_t f, uint32_t S[12]) {
  uint32_t i, j, k;
  const int o = face_pos(G, f, i, j, k);
#pragma unroll
  for (int q = 0; q < 12; ++q) S[q] = 0xFFFFFFFFu;
  auto fill = [&](auto lc, uint32_t, const uint32_t F[6], uint32_t) {
    constexpr int side = (decltype(lc)::value & 1) ? 0 : 1;
#pragma unroll
    for (int e = 0; e < 6; ++e) S[6 * side + e] = F[e];
  };
  if (o == 0)
    visit_face_cells<0>(G, i, j, k, fill);
  else if (o == 1)
    visit_face_cells<1>(G, i, j, k, fill);
  else
    visit_face_cells<2>(G, i, j, k, fill);
}

__global__ void k_mask_faces(Grid G, const int* __restrict__ rp, const int* __restrict__ col,
                             const uint8_t* __restrict__ strong, uint32_t* __restrict__ mask, int* __restrict__ bad) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= G.nf) return;
  uint32_t S[12];
  face_slots(G, (uint32_t)f, S);
  uint32_t m = 0;
  for (int e = rp[f]; e < rp[f + 1]; ++e) {
    if (strong[e] != 1) continue;
    const uint32_t g = (uint32_t)col[e];
    uint32_t hit = 0;
#pragma unroll
    for (int q = 0; q < 12; ++q) hit |= (S[q] == g ? 1u : 0u) << q;
    if (!hit) *bad = 1;
    m |= hit;
  }
  mask[f] = m;
}

__global__ void __launch_bounds__(256) k_mis_max_faces(Grid G, const uint32_t* __restrict__ mask,
                                                       const uint64_t* __restrict__ Tin,
                                                       uint64_t* __restrict__ Tout, const int* __restrict__ go) {
  if (!*go) return;
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= G.nf) return;
  const uint32_t bits = mask[f];
  uint64_t m = Tin[f];
  if (bits) {
    uint32_t S[12];
    face_slots(G, (uint32_t)f, S);
#pragma unroll
    for (int q = 0; q < 12; ++q) {
      if (!((bits >> q) & 1u)) continue;
      const uint64_t v = ld32(Tin, S[q]);
      m = v > m ? v : m;
    }
  }
  Tout[f] = m;
}

__global__ void k_mis_update(int n, const uint64_t* __restrict__ T0, const uint64_t* __restrict__ T2,
                             uint8_t* __restrict__ state, int* __restrict__ und, const int* __restrict__ go) {
  if (!*go) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  bool left = false;
  if (state[i] == kUnd) {
    if (T2[i] == T0[i]) {
      state[i] = kIn;
    } else if ((T2[i] >> 62) == 2) {
      state[i] = kOut;
    } else {
      left = true;
    }
  }
  // one flag store per wavefront with undecided rows
  const unsigned long long m = __ballot(left);
  if (m != 0ull && (threadIdx.x & 63) == (unsigned)(__ffsll((long long)m) - 1)) *und = 1;
}

__global__ void k_root_flags(int n, const uint8_t* __restrict__ state, int* __restrict__ f) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) f[i] = state[i] == kIn;
}

// distance-1 attachment: a node joins its most strongly coupled root
template <int BS, int G>
__global__ void __launch_bounds__(256) k_agg_phase1(int n, const int* __restrict__ rp, const int* __restrict__ col,
                                                    BlockNorms<BS> nv, const uint8_t* __restrict__ strong,
                                                    const uint8_t* __restrict__ state,
                                                    const int* __restrict__ root_id, int* __restrict__ agg1) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = (int)(t / G), l = (int)(t % G);
  int a = -1, eb = INT_MAX;
  double best = -1.0;
  const bool root = i < n && state[i] == kIn;
  if (i < n && !root)
    for (int e = rp[i] + l; e < rp[i + 1]; e += G)
      if (strong[e] == 1 && state[col[e]] == kIn) {
        const double sv = nv(e);
        if (sv > best) {
          best = sv;
          eb = e;
          a = root_id[col[e]];
        }
      }
  argmax_lanes<G>(best, eb, a);
  if (i < n && l == 0) agg1[i] = root ? root_id[i] : a;
}

template <int BS, int G>
__global__ void __launch_bounds__(256) k_agg_phase2(int n, const int* __restrict__ rp, const int* __restrict__ col,
                                                    BlockNorms<BS> nv, const uint8_t* __restrict__ strong,
                                                    const int* __restrict__ agg1, int* __restrict__ agg,
                                                    int* __restrict__ status) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = (int)(t / G), l = (int)(t % G);
  const int a1 = i < n ? agg1[i] : 0;
  int a = -1, eb = INT_MAX, has_strong = 0;
  double best = -1.0;
  if (i < n && a1 < 0)
    for (int e = rp[i] + l; e < rp[i + 1]; e += G) {
      if (strong[e] != 1) continue;
      has_strong = 1;
      const int j = col[e];
      if (agg1[j] < 0) continue;
      const double sv = nv(e);
      if (sv > best) {
        best = sv;
        eb = e;
        a = agg1[j];
      }
    }
  argmax_lanes<G>(best, eb, a);
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) has_strong |= __shfl_xor(has_strong, o, G);
  if (i < n && l == 0) {
    if (a1 >= 0) {
      agg[i] = a1;
    } else {
      if (has_strong && a < 0) atomicOr(status, kStatusCapacity);
      agg[i] = a;
    }
  }
}

__global__ void k_count_aggregated(int n, const int* __restrict__ agg, int* __restrict__ f) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) f[i] = agg[i] >= 0;
}

template <int BS>
__global__ void k_ptent(int n, const int* __restrict__ agg, const int* __restrict__ rp, int* __restrict__ col,
                        double* __restrict__ val) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || agg[i] < 0) return;
  const int e = rp[i];
  col[e] = agg[i];
  for (int a = 0; a < BS; ++a)
    for (int b = 0; b < BS; ++b) val[(size_t)e * BS * BS + a * BS + b] = a == b ? 1.0 : 0.0;
}

// P = P_tent - omega D^-1 (A P_tent), in place on the pattern of A P_tent
template <int BS>
__global__ void k_smooth_p(int n, const int* __restrict__ agg, const double* __restrict__ dinv, double omega,
                           const int* __restrict__ rp, const int* __restrict__ col, double* __restrict__ val) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double* D = dinv + (size_t)i * BS * BS;
  for (int e = rp[i]; e < rp[i + 1]; ++e) {
    double* v = val + (size_t)e * BS * BS;
    double o[BS * BS];
    for (int a = 0; a < BS; ++a)
      for (int b = 0; b < BS; ++b) {
        double s = 0.0;
        for (int t = 0; t < BS; ++t) s += D[a * BS + t] * v[t * BS + b];
        o[a * BS + b] = -omega * s + ((col[e] == agg[i] && a == b) ? 1.0 : 0.0);
      }
    for (int q = 0; q < BS * BS; ++q) v[q] = o[q];
  }
}

// Truncation of a prolongator: blocks whose norm is below tau * (largest block
// norm of the row) are dropped and the kept ones rescaled so that the row's
// block sum is unchanged (scalar: by the ratio of sums; 3x3: right-multiplied
// by (sum kept)^-1 (sum all)), so that interpolation of the near kernel
// (constants, or rigid translations per component) is unchanged.
template <int BS>
__device__ inline double pblock_norm(const double* v) {
  double s = 0.0;
  for (int q = 0; q < BS * BS; ++q) s += v[q] * v[q];
  return sqrt(s);
}

// rigid-body prolongators (rigid = true): translation (even) and rotation
// (odd) columns have different units, so each block is compared with the
// largest of its own kind in the row, and nothing is rescaled
template <int BS>
__device__ inline void trunc_row_max(int i, const int* __restrict__ rp, const int* __restrict__ col,
                                     const double* __restrict__ val, bool rigid, double mx[2]) {
  mx[0] = mx[1] = 0.0;
  for (int e = rp[i]; e < rp[i + 1]; ++e) {
    const int k = rigid ? (col[e] & 1) : 0;
    mx[k] = fmax(mx[k], pblock_norm<BS>(val + (size_t)e * BS * BS));
  }
}

template <int BS>
__device__ inline bool trunc_keep(int e, const int* __restrict__ col, const double* __restrict__ val, bool rigid,
                                  double tau, const double mx[2]) {
  return pblock_norm<BS>(val + (size_t)e * BS * BS) >= tau * mx[rigid ? (col[e] & 1) : 0];
}

template <int BS>
__global__ void k_trunc_count(int n, const int* __restrict__ rp, const int* __restrict__ col,
                              const double* __restrict__ val, double tau, bool rigid, int* __restrict__ cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double mx[2];
  trunc_row_max<BS>(i, rp, col, val, rigid, mx);
  int c = 0;
  for (int e = rp[i]; e < rp[i + 1]; ++e) c += trunc_keep<BS>(e, col, val, rigid, tau, mx);
  cnt[i] = c;
}

template <int BS>
__global__ void k_trunc_fill(int n, const int* __restrict__ rp, const int* __restrict__ col,
                             const double* __restrict__ val, double tau, bool rigid, const int* __restrict__ trp,
                             int* __restrict__ tcol, double* __restrict__ tval) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double mx[2], all[BS * BS], kept[BS * BS];
  trunc_row_max<BS>(i, rp, col, val, rigid, mx);
  for (int q = 0; q < BS * BS; ++q) all[q] = kept[q] = 0.0;
  for (int e = rp[i]; e < rp[i + 1]; ++e) {
    const double* v = val + (size_t)e * BS * BS;
    for (int q = 0; q < BS * BS; ++q) all[q] += v[q];
    if (trunc_keep<BS>(e, col, val, rigid, tau, mx))
      for (int q = 0; q < BS * BS; ++q) kept[q] += v[q];
  }
  // S = kept^-1 all (identity if kept is singular)
  double S[BS * BS];
  for (int q = 0; q < BS * BS; ++q) S[q] = (q % (BS + 1) == 0) ? 1.0 : 0.0;
  if (rigid) {
  } else if (BS == 1) {
    if (kept[0] != 0.0) S[0] = all[0] / kept[0];
  } else {
    const double* k = kept;
    const double det = k[0] * (k[4] * k[8] - k[5] * k[7]) - k[1] * (k[3] * k[8] - k[5] * k[6]) +
                       k[2] * (k[3] * k[7] - k[4] * k[6]);
    if (det != 0.0 && isfinite(det)) {
      double inv[9];
      inv[0] = (k[4] * k[8] - k[5] * k[7]) / det;
      inv[1] = (k[2] * k[7] - k[1] * k[8]) / det;
      inv[2] = (k[1] * k[5] - k[2] * k[4]) / det;
      inv[3] = (k[5] * k[6] - k[3] * k[8]) / det;
      inv[4] = (k[0] * k[8] - k[2] * k[6]) / det;
      inv[5] = (k[2] * k[3] - k[0] * k[5]) / det;
      inv[6] = (k[3] * k[7] - k[4] * k[6]) / det;
      inv[7] = (k[1] * k[6] - k[0] * k[7]) / det;
      inv[8] = (k[0] * k[4] - k[1] * k[3]) / det;
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          double t = 0.0;
          for (int c = 0; c < 3; ++c) t += inv[a * 3 + c] * all[c * 3 + b];
          S[a * 3 + b] = t;
        }
    }
  }
  int p = trp[i];
  for (int e = rp[i]; e < rp[i + 1]; ++e) {
    const double* v = val + (size_t)e * BS * BS;
    if (!trunc_keep<BS>(e, col, val, rigid, tau, mx)) continue;
    tcol[p] = col[e];
    for (int a = 0; a < BS; ++a)
      for (int b = 0; b < BS; ++b) {
        double t = 0.0;
        for (int c = 0; c < BS; ++c) t += v[a * BS + c] * S[c * BS + b];
        tval[(size_t)p * BS * BS + a * BS + b] = t;
      }
    ++p;
  }
}

template <int BS>
void truncate_p(hipStream_t s, Csr& P, double tau, bool rigid = false) {
  int* cnt = dalloc<int>(P.n);
  k_trunc_count<BS><<<blocks_for(P.n), kBlock, 0, s>>>(P.n, P.rowptr, P.col, P.val, tau, rigid, cnt);
  PM_CHECK_LAUNCH();
  Csr T;
  T.bs = BS;
  T.n = P.n;
  T.m = P.m;
  T.rowptr = dalloc<int>(P.n + 1);
  int nnz = 0;
  exclusive_scan(s, cnt, T.rowptr, P.n, &nnz);
  dfree(cnt);
  T.nnzb = nnz;
  T.col = dalloc<int>(nnz);
  T.val = dalloc<double>((int64_t)nnz * BS * BS);
  k_trunc_fill<BS><<<blocks_for(P.n), kBlock, 0, s>>>(P.n, P.rowptr, P.col, P.val, tau, rigid, T.rowptr, T.col,
                                                      T.val);
  PM_CHECK_LAUNCH();
  P.free_all();
  P = T;
}

// filtered operator for prolongator smoothing: strong off-diagonal blocks
// kept, weak ones lumped into the diagonal block (row sums preserved)
// entries kept in A_F (diagonal and strong); *any_weak is set when some row
// drops a nonzero block.  G lanes per row as in the strength kernels.
template <int G>
__global__ void __launch_bounds__(256) k_filter_count(int n, const int* __restrict__ rp,
                                                      const int* __restrict__ col,
                                                      const uint8_t* __restrict__ strong, int* __restrict__ cnt,
                                                      int* __restrict__ any_weak) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = (int)(t / G), l = (int)(t % G);
  int c = 0, w = 0;
  if (i < n)
    for (int e = rp[i] + l; e < rp[i + 1]; e += G) {
      const bool diag = col[e] == i;
      c += diag || strong[e] == 1;
      w |= !diag && strong[e] == 0;
    }
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) c += __shfl_xor(c, o, G);
  if (i < n && l == 0) cnt[i] = c;
  // one flag store per wavefront that has a weak coupling (all store 1)
  const unsigned long long m = __ballot(w != 0);
  if (m != 0ull && (threadIdx.x & 63) == (unsigned)(__ffsll((long long)m) - 1)) *any_weak = 1;
}

// A_F rows: the kept entries in their order, the weak blocks summed (lane
// partial sums, then a shuffle tree) onto the diagonal block
template <int BS, int G>
__global__ void __launch_bounds__(256) k_filter_fill(int n, const int* __restrict__ rp, const int* __restrict__ col,
                                                     const double* __restrict__ val,
                                                     const uint8_t* __restrict__ strong,
                                                     const int* __restrict__ frp, int* __restrict__ fcol,
                                                     double* __restrict__ fval) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = (int)(t / G), l = (int)(t % G);
  double lump[BS * BS];
#pragma unroll
  for (int q = 0; q < BS * BS; ++q) lump[q] = 0.0;
  const int e0 = i < n ? rp[i] : 0, e1 = i < n ? rp[i + 1] : 0;
  for (int e = e0 + l; e < e1; e += G)
    if (col[e] != i && strong[e] == 0)
#pragma unroll
      for (int q = 0; q < BS * BS; ++q) lump[q] += val[(size_t)e * BS * BS + q];
#pragma unroll
  for (int q = 0; q < BS * BS; ++q)
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) lump[q] += __shfl_xor(lump[q], o, G);
  // compaction: each pass over G entries places the kept ones after those of
  // the lower lanes (ballot of the row's lane group)
  const int lane = threadIdx.x & 63, base = lane & ~(G - 1);
  const unsigned long long gmask = (G == 64) ? ~0ull : ((1ull << G) - 1ull);
  int p = i < n ? frp[i] : 0;
  for (int e00 = e0; e00 < e1; e00 += G) {  // same trip count on every lane of the row
    const int e = e00 + l;
    const bool diag = e < e1 && col[e] == i;
    const bool keep = e < e1 && (diag || strong[e] == 1);
    const unsigned long long grp = (__ballot(keep) >> base) & gmask;
    if (keep) {
      const int q0 = p + __popcll(grp & ((1ull << l) - 1ull));
      fcol[q0] = col[e];
#pragma unroll
      for (int q = 0; q < BS * BS; ++q)
        fval[(size_t)q0 * BS * BS + q] = val[(size_t)e * BS * BS + q] + (diag ? lump[q] : 0.0);
    }
    p += __popcll(grp);
  }
}

// ---------------------------------------------------------------------------
// deterministic reductions (sum of squares), two stages
constexpr int kRedBlocks = 1024;

template <class T>
__global__ void __launch_bounds__(256) k_sumsq_part(const T* __restrict__ x, int64_t n, double* __restrict__ part) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double v = (double)x[i];
    s += v * v;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(256) k_sum_final(const double* __restrict__ part, int np, double* __restrict__ out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) s += part[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

template <class T>
__global__ void k_rand_vec(int64_t n, T* __restrict__ x, uint32_t salt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = (T)((double)(mix32((uint32_t)i ^ salt) & 0xFFFFFF) / 16777216.0 + 0.5);
}

// One power-iteration step after the operator product w = A v: nsq = the sum
// of the previous step's partial sums (in k_sum_final's order), v = D^-1 w /
// sqrt(nsq), and this step's partial sums of v^2 (in k_sumsq_part's order,
// so with kRedBlocks workgroups the iterates equal those of the separate
// kernels bit for bit).  TV: the iterates (double, or float on the FP32
// operators), TD: the block-diagonal inverse; products and sums in FP64.
template <int BS, class TV, class TD>
__global__ void __launch_bounds__(256) k_power_step(int64_t n, const TD* __restrict__ dinv,
                                                    const TV* __restrict__ w, const double* __restrict__ part_in,
                                                    TV* __restrict__ v, double* __restrict__ part_out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < kRedBlocks; i += 256) s += part_in[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  const double q = sh[0];
  __syncthreads();
  const double scale = q > 0.0 ? 1.0 / sqrt(q) : 0.0;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const int64_t node = i / BS;
    const int a = (int)(i - node * BS);
    const TD* D = dinv + (size_t)node * BS * BS + a * BS;
    double t = 0.0;
    for (int b = 0; b < BS; ++b) t += (double)D[b] * (double)w[(size_t)node * BS + b];
    const TV x = (TV)(t * scale);
    v[i] = x;
    acc += (double)x * (double)x;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part_out[blockIdx.x] = sh[0];
}

// ---------------------------------------------------------------------------
// cycle kernels (T = double or float)
template <int BS, class T>
__device__ inline void dinv_mul(const T* __restrict__ D, const T r[BS], T out[BS]) {
  for (int a = 0; a < BS; ++a) {
    T s = 0;
    for (int b = 0; b < BS; ++b) s += D[a * BS + b] * r[b];
    out[a] = s;
  }
}

// first Chebyshev step from x = 0: d = D^-1 b / theta, x = d
template <int BS, class T>
__global__ void k_cheb_first(int n, const T* __restrict__ dinv, const T* __restrict__ b, T inv_theta,
                             T* __restrict__ x, T* __restrict__ d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T bi[BS], z[BS];
  for (int a = 0; a < BS; ++a) bi[a] = b[(size_t)i * BS + a];
  dinv_mul<BS, T>(dinv + (size_t)i * BS * BS, bi, z);
  for (int a = 0; a < BS; ++a) {
    const T v = z[a] * inv_theta;
    d[(size_t)i * BS + a] = v;
    x[(size_t)i * BS + a] = v;
  }
}

// fused step: r = D^-1 (b - A x_in); d = c1 d + c2 r; x_out = x_in + d
template <int BS, class T>
__global__ void __launch_bounds__(256) k_cheb_step(int n, const int* __restrict__ sptr,
                                                   const int* __restrict__ perm, const int* __restrict__ col,
                                                   const T* __restrict__ val, const T* __restrict__ dinv,
                                                   const T* __restrict__ b, const T* __restrict__ xin,
                                                   T* __restrict__ xout, T* __restrict__ d, T c1, T c2) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = t / kSlice, lane = t % kSlice;
  if (s * kSlice >= n) return;
  const int e0 = sptr[s], e1 = sptr[s + 1];
  T acc[BS];
  for (int q = 0; q < BS; ++q) acc[q] = 0;
  sell_row<BS, SellUnroll<BS>::value, T, T>(e0, e1, col, val, xin, lane, acc);
  const int r = sell_row_of(perm, t, n);
  if (r < 0) return;
  T res[BS], z[BS];
  for (int a = 0; a < BS; ++a) res[a] = b[(size_t)r * BS + a] - acc[a];
  dinv_mul<BS, T>(dinv + (size_t)r * BS * BS, res, z);
  for (int a = 0; a < BS; ++a) {
    const size_t k = (size_t)r * BS + a;
    const T dn = c1 * d[k] + c2 * z[a];
    d[k] = dn;
    xout[k] = xin[k] + dn;
  }
}

// residual r = b - A x
template <int BS, class T>
__global__ void __launch_bounds__(256) k_residual(int n, const int* __restrict__ sptr,
                                                  const int* __restrict__ perm, const int* __restrict__ col,
                                                  const T* __restrict__ val, const T* __restrict__ b,
                                                  const T* __restrict__ x, T* __restrict__ rr) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = t / kSlice, lane = t % kSlice;
  if (s * kSlice >= n) return;
  const int e0 = sptr[s], e1 = sptr[s + 1];
  T acc[BS];
  for (int q = 0; q < BS; ++q) acc[q] = 0;
  sell_row<BS, SellUnroll<BS>::value, T, T>(e0, e1, col, val, x, lane, acc);
  const int r = sell_row_of(perm, t, n);
  if (r < 0) return;
  for (int a = 0; a < BS; ++a) rr[(size_t)r * BS + a] = b[(size_t)r * BS + a] - acc[a];
}

// y = A x (ADD = false) or y += A x (ADD = true): restriction and prolongation
template <int BS, class T, bool ADD>
__global__ void __launch_bounds__(256) k_sell_apply(int n, const int* __restrict__ sptr,
                                                    const int* __restrict__ perm, const int* __restrict__ col,
                                                    const T* __restrict__ val, const T* __restrict__ xc,
                                                    T* __restrict__ x) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = t / kSlice, lane = t % kSlice;
  if (s * kSlice >= n) return;
  const int e0 = sptr[s], e1 = sptr[s + 1];
  T acc[BS];
  for (int q = 0; q < BS; ++q) acc[q] = 0;
  sell_row<BS, SellUnroll<BS>::value, T, T>(e0, e1, col, val, xc, lane, acc);
  const int r = sell_row_of(perm, t, n);
  if (r < 0) return;
  for (int a = 0; a < BS; ++a) {
    if (ADD)
      x[(size_t)r * BS + a] += acc[a];
    else
      x[(size_t)r * BS + a] = acc[a];
  }
}

// Levels with long rows (coarse Galerkin operators): G lanes per block row
// stride over its CSR entries, the partial sums are combined with a fixed
// xor tree (deterministic), and lane a < BS finishes component a.
template <int BS, class T, int G>
__device__ inline void csr_row_lanes(int row, int lane, const int* __restrict__ rp, const int* __restrict__ col,
                                     const T* __restrict__ val, const T* __restrict__ x, T acc[BS]) {
  for (int a = 0; a < BS; ++a) acc[a] = 0;
  const int e1 = rp[row + 1];
  int e = rp[row] + lane;
  // two entries of the lane per step, both loaded before either is summed
  // (the same order of summation as one at a time)
  for (; e + G < e1; e += 2 * G) {
    const int j0 = col[e], j1 = col[e + G];
    T v0[BS * BS], v1[BS * BS], x0[BS], x1[BS];
    for (int q = 0; q < BS * BS; ++q) {
      v0[q] = val[(size_t)e * BS * BS + q];
      v1[q] = val[(size_t)(e + G) * BS * BS + q];
    }
    for (int q = 0; q < BS; ++q) {
      x0[q] = x[(size_t)j0 * BS + q];
      x1[q] = x[(size_t)j1 * BS + q];
    }
    for (int a = 0; a < BS; ++a)
      for (int q = 0; q < BS; ++q) acc[a] += v0[a * BS + q] * x0[q];
    for (int a = 0; a < BS; ++a)
      for (int q = 0; q < BS; ++q) acc[a] += v1[a * BS + q] * x1[q];
  }
  if (e < e1) {
    const int j = col[e];
    const T* v = val + (size_t)e * BS * BS;
    T xj[BS];
    for (int q = 0; q < BS; ++q) xj[q] = x[(size_t)j * BS + q];
    for (int a = 0; a < BS; ++a)
      for (int q = 0; q < BS; ++q) acc[a] += v[a * BS + q] * xj[q];
  }
}

template <int BS, class T, int G>
__device__ inline void lanes_reduce(T acc[BS]) {
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1)
    for (int a = 0; a < BS; ++a) acc[a] += __shfl_xor(acc[a], off, G);
}

// Chebyshev step on a CSR level: r = D^-1 (b - A x_in); d = c1 d + c2 r; x_out = x_in + d
template <int BS, class T, int G>
__global__ void __launch_bounds__(256) k_cheb_step_csr(int n, const int* __restrict__ rp, const int* __restrict__ col,
                                                       const T* __restrict__ val, const T* __restrict__ dinv,
                                                       const T* __restrict__ b, const T* __restrict__ xin,
                                                       T* __restrict__ xout, T* __restrict__ d, T c1, T c2) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int row = (int)(t / G), lane = (int)(t % G);
  T acc[BS];
  if (row < n)
    csr_row_lanes<BS, T, G>(row, lane, rp, col, val, xin, acc);
  else
    for (int a = 0; a < BS; ++a) acc[a] = 0;
  lanes_reduce<BS, T, G>(acc);
  if (row >= n || lane >= BS) return;
  T res[BS];
  for (int a = 0; a < BS; ++a) res[a] = b[(size_t)row * BS + a] - acc[a];
  T z = 0;
  for (int q = 0; q < BS; ++q) z += dinv[(size_t)row * BS * BS + lane * BS + q] * res[q];
  const size_t k = (size_t)row * BS + lane;
  const T dn = c1 * d[k] + c2 * z;
  d[k] = dn;
  xout[k] = xin[k] + dn;
}

// residual r = b - A x (RES) or product r = A x on a CSR level
template <int BS, class T, int G, bool RES>
__global__ void __launch_bounds__(256) k_residual_csr(int n, const int* __restrict__ rp, const int* __restrict__ col,
                                                      const T* __restrict__ val, const T* __restrict__ b,
                                                      const T* __restrict__ x, T* __restrict__ rr) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int row = (int)(t / G), lane = (int)(t % G);
  T acc[BS];
  if (row < n)
    csr_row_lanes<BS, T, G>(row, lane, rp, col, val, x, acc);
  else
    for (int a = 0; a < BS; ++a) acc[a] = 0;
  lanes_reduce<BS, T, G>(acc);
  if (row >= n || lane >= BS) return;
  T v = acc[0];
  for (int a = 1; a < BS; ++a)
    if (lane == a) v = acc[a];
  rr[(size_t)row * BS + lane] = RES ? b[(size_t)row * BS + lane] - v : v;
}

// launch the CSR-lane kernels with G in {4, 8, 16} lanes per row
template <int BS, class T>
void cheb_step_csr(hipStream_t s, const Level& L, const T* val, const T* dinv, const T* b, const T* xin, T* xout,
                   T* d, T c1, T c2) {
  const int n = L.n;
  switch (L.csr_lanes) {
    case 4:
      k_cheb_step_csr<BS, T, 4><<<blocks_for((int64_t)n * 4), kBlock, 0, s>>>(n, L.A.rowptr, L.A.col, val, dinv, b,
                                                                              xin, xout, d, c1, c2);
      break;
    case 8:
      k_cheb_step_csr<BS, T, 8><<<blocks_for((int64_t)n * 8), kBlock, 0, s>>>(n, L.A.rowptr, L.A.col, val, dinv, b,
                                                                              xin, xout, d, c1, c2);
      break;
    default:
      k_cheb_step_csr<BS, T, 16><<<blocks_for((int64_t)n * 16), kBlock, 0, s>>>(n, L.A.rowptr, L.A.col, val, dinv,
                                                                                b, xin, xout, d, c1, c2);
  }
  PM_CHECK_LAUNCH();
}

template <int BS, class T, bool RES>
void residual_csr(hipStream_t s, const Csr& A, int lanes, const T* val, const T* b, const T* x, T* r) {
  const int n = A.n;
  switch (lanes) {
    case 4:
      k_residual_csr<BS, T, 4, RES><<<blocks_for((int64_t)n * 4), kBlock, 0, s>>>(n, A.rowptr, A.col, val, b, x, r);
      break;
    case 8:
      k_residual_csr<BS, T, 8, RES><<<blocks_for((int64_t)n * 8), kBlock, 0, s>>>(n, A.rowptr, A.col, val, b, x, r);
      break;
    case 64:
      k_residual_csr<BS, T, 64, RES><<<blocks_for((int64_t)n * 64), kBlock, 0, s>>>(n, A.rowptr, A.col, val, b, x,
                                                                                    r);
      break;
    default:
      k_residual_csr<BS, T, 16, RES><<<blocks_for((int64_t)n * 16), kBlock, 0, s>>>(n, A.rowptr, A.col, val, b, x,
                                                                                    r);
  }
  PM_CHECK_LAUNCH();
}

// lanes per row, 4 to 16: about a quarter of the average row length for
// scalar rows, about half of it for 3x3 blocks (nine values per entry)
inline int csr_lanes_for(const Csr& A) {
  const double avg = (double)A.nnzb / std::max(1, A.n);
  if (A.bs == 3) return avg < 12.0 ? 4 : (avg < 24.0 ? 8 : 16);
  return avg < 24.0 ? 4 : (avg < 48.0 ? 8 : 16);
}
// restrictions P^T have few, long rows on the coarse levels: a wavefront per
// row once rows average 128 blocks or more
inline int restrict_lanes_for(const Csr& R) {
  const double avg = (double)R.nnzb / std::max(1, R.n);
  return avg >= 128.0 ? 64 : csr_lanes_for(R);
}

// dense coarse level
__global__ void k_dense_from_csr(int nb, int bs, const int* __restrict__ rp, const int* __restrict__ col,
                                 const double* __restrict__ val, double* __restrict__ M, int ld) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  for (int e = rp[i]; e < rp[i + 1]; ++e)
    for (int a = 0; a < bs; ++a)
      for (int b = 0; b < bs; ++b)
        M[(size_t)(i * bs + a) * ld + (size_t)col[e] * bs + b] = val[(size_t)e * bs * bs + a * bs + b];
}

__global__ void k_set_identity_right(int n, double* __restrict__ M) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) M[(size_t)i * 2 * n + n + i] = 1.0;
}

// Gauss-Jordan step k, part 1: save column k, scale row k by its pivot
__global__ void __launch_bounds__(256) k_gj_pivot(int n, int k, double* __restrict__ M, double* __restrict__ colk,
                                                  int* __restrict__ status) {
  __shared__ double piv;
  if (threadIdx.x == 0) {
    piv = M[(size_t)k * 2 * n + k];
    if (!(piv > 0.0)) atomicOr(status, kStatusBadPivot);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) colk[i] = (i == k) ? 0.0 : M[(size_t)i * 2 * n + k];
  __syncthreads();
  const double r = 1.0 / piv;
  for (int j = threadIdx.x; j < 2 * n; j += blockDim.x) M[(size_t)k * 2 * n + j] *= r;
}

// part 2: eliminate column k from all other rows
__global__ void k_gj_elim(int n, int k, double* __restrict__ M, const double* __restrict__ colk) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t w = 2 * (int64_t)n;
  if (t >= (int64_t)n * w) return;
  const int i = (int)(t / w), j = (int)(t % w);
  if (i == k) return;
  M[t] -= colk[i] * M[(size_t)k * w + j];
}

// All n Gauss-Jordan steps in one workgroup, inverting in place in LDS (n^2
// doubles; no pivoting, the coarsest operators are SPD): one launch instead
// of 2n.  Reads the left half of the augmented matrix and writes the inverse
// into its right half, where k_extract_inverse expects it.
constexpr int kGjLdsBytes = 160 * 1024;
constexpr int kGjMaxN = 256;
__global__ void __launch_bounds__(1024) k_gj_lds(int n, double* __restrict__ M, int* __restrict__ status) {
  extern __shared__ double S[];
  __shared__ double rowk[kGjMaxN], colk[kGjMaxN];
  __shared__ double piv;
  const int nn = n * n;
  for (int t = threadIdx.x; t < nn; t += blockDim.x) S[t] = M[(size_t)(t / n) * 2 * n + (t % n)];
  const int i0 = (int)threadIdx.x / n, j0 = (int)threadIdx.x % n;
  const int di = (int)blockDim.x / n, dj = (int)blockDim.x % n;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (threadIdx.x == 0) {
      piv = S[k * n + k];
      if (!(piv > 0.0)) atomicOr(status, kStatusBadPivot);
    }
    __syncthreads();
    const double p = 1.0 / piv;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
      rowk[j] = (j == k) ? p : S[k * n + j] * p;
      colk[j] = (j == k) ? 0.0 : S[j * n + k];
    }
    __syncthreads();
    // (i, j) of t advanced without division: t grows by blockDim.x each pass
    int i = i0, j = j0;
    for (int t = threadIdx.x; t < nn; t += blockDim.x) {
      if (i == k)
        S[t] = rowk[j];
      else if (j == k)
        S[t] = -colk[i] * p;
      else
        S[t] -= colk[i] * rowk[j];
      i += di;
      j += dj;
      if (j >= n) {
        j -= n;
        ++i;
      }
    }
    __syncthreads();
  }
  for (int t = threadIdx.x; t < nn; t += blockDim.x) M[(size_t)(t / n) * 2 * n + n + (t % n)] = S[t];
}

__global__ void k_extract_inverse(int n, const double* __restrict__ M, double* __restrict__ inv) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * n) return;
  const int i = (int)(t / n), j = (int)(t % n);
  const double a = M[(size_t)i * 2 * n + n + j], b = M[(size_t)j * 2 * n + n + i];
  inv[t] = 0.5 * (a + b);
}

// y = Ainv x (one wavefront per row; x may be float or double)
template <class T>
__global__ void __launch_bounds__(256) k_dense_gemv(int n, const double* __restrict__ Ainv, const T* __restrict__ x,
                                                    T* __restrict__ y) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (row >= n) return;
  double s = 0.0;
  for (int j = lane; j < n; j += 64) s += Ainv[(size_t)row * n + j] * (double)x[j];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) y[row] = (T)s;
}

__global__ void k_to_float(int64_t n, const double* __restrict__ a, float* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

template <int BS>
void launch_cheb_first(hipStream_t s, int n, const double* dinv, const double* b, double it, double* x, double* d) {
  k_cheb_first<BS, double><<<blocks_for(n), kBlock, 0, s>>>(n, dinv, b, it, x, d);
}
template <int BS>
void launch_cheb_first(hipStream_t s, int n, const float* dinv, const float* b, float it, float* x, float* d) {
  k_cheb_first<BS, float><<<blocks_for(n), kBlock, 0, s>>>(n, dinv, b, it, x, d);
}

// ---------------------------------------------------------------------------
double sum_squares(hipStream_t s, const double* x, int64_t n, double* part, double* out_dev) {
  k_sumsq_part<double><<<kRedBlocks, 256, 0, s>>>(x, n, part);
  k_sum_final<<<1, 256, 0, s>>>(part, kRedBlocks, out_dev);
  double h = 0.0;
  PM_HIP(hipMemcpyAsync(&h, out_dev, sizeof(double), hipMemcpyDeviceToHost, s));
  PM_HIP(hipStreamSynchronize(s));
  return h;
}

// lambda_max(D^-1 A) by power iteration from a fixed pseudo-random start;
// spmv(stream, v, w) launches w = A v on the stream.  The iteration can run
// on a second stream while the caller's stream goes on (power_start /
// power_finish): it reads only the operator and D^-1, which the caller keeps
// unchanged until the result is taken, and the result does not depend on the
// stream.
struct PowerJob {
  hipStream_t s2 = nullptr;
  hipEvent_t ready = nullptr, done = nullptr;
  double *v = nullptr, *w = nullptr, *pbuf = nullptr, *nsq = nullptr;
  bool pending() const { return s2 != nullptr; }
  PowerJob() = default;
  PowerJob(const PowerJob&) = delete;
  PowerJob& operator=(const PowerJob&) = delete;
  PowerJob& operator=(PowerJob&& o) noexcept {
    std::swap(s2, o.s2);
    std::swap(ready, o.ready);
    std::swap(done, o.done);
    std::swap(v, o.v);
    std::swap(w, o.w);
    std::swap(pbuf, o.pbuf);
    std::swap(nsq, o.nsq);
    return *this;
  }
  void release() {
    if (s2) (void)hipStreamSynchronize(s2);  // the buffers are in use until the stream drains
    for (double* p : {v, w, pbuf, nsq}) dfree(p);
    if (ready) (void)hipEventDestroy(ready);
    if (done) (void)hipEventDestroy(done);
    s2 = nullptr;
    ready = done = nullptr;
    v = w = pbuf = nsq = nullptr;
  }
  ~PowerJob() { release(); }
};

// the job's vectors hold n doubles, or n floats when the iteration runs on
// the FP32 copies of the operator (TV = float)
template <class TV, class TD, class F>
void power_launch(hipStream_t s, const PowerJob& j, int64_t nb, int bs, const TD* dinv, int its, F spmv) {
  const int64_t n = nb * bs;
  double *part = j.pbuf, *part2 = j.pbuf + kRedBlocks;
  TV* v = reinterpret_cast<TV*>(j.v);
  TV* w = reinterpret_cast<TV*>(j.w);
  k_rand_vec<TV><<<blocks_for(n), kBlock, 0, s>>>(n, v, 0x9e3779b9u);
  // ||v|| stays on the device: lambda ~ ||D^-1 A v|| / ||v|| with v normalised
  k_sumsq_part<TV><<<kRedBlocks, 256, 0, s>>>(v, n, part);
  for (int k = 0; k < its; ++k) {
    spmv(s, v, w);
    if (bs == 3)
      k_power_step<3, TV, TD><<<kRedBlocks, 256, 0, s>>>(n, dinv, w, part, v, part2);
    else
      k_power_step<1, TV, TD><<<kRedBlocks, 256, 0, s>>>(n, dinv, w, part, v, part2);
    std::swap(part, part2);
  }
  k_sum_final<<<1, 256, 0, s>>>(part, kRedBlocks, j.nsq);
  PM_CHECK_LAUNCH();
}

void power_alloc(PowerJob& j, int64_t n) {
  j.v = dalloc<double>(n);
  j.w = dalloc<double>(n);
  j.pbuf = dalloc<double>(2 * kRedBlocks);
  j.nsq = dalloc<double>(1);
}

template <class TV = double, class TD = double, class F>
double power_lmax(hipStream_t s, int64_t nb, int bs, const TD* dinv, int its, F spmv) {
  PowerJob j;
  power_alloc(j, nb * bs);
  power_launch<TV>(s, j, nb, bs, dinv, its, spmv);
  double h = 0.0;
  PM_HIP(hipMemcpyAsync(&h, j.nsq, sizeof(double), hipMemcpyDeviceToHost, s));
  PM_HIP(hipStreamSynchronize(s));
  return std::sqrt(h);
}

// the same on stream s2, after the work queued so far on s
template <class TV = double, class TD = double, class F>
void power_start(PowerJob& j, hipStream_t s, hipStream_t s2, int64_t nb, int bs, const TD* dinv, int its,
                 F spmv) {
  j.release();
  power_alloc(j, nb * bs);
  j.s2 = s2;
  PM_HIP(hipEventCreateWithFlags(&j.ready, hipEventDisableTiming));
  PM_HIP(hipEventCreateWithFlags(&j.done, hipEventDisableTiming));
  PM_HIP(hipEventRecord(j.ready, s));
  PM_HIP(hipStreamWaitEvent(s2, j.ready, 0));
  power_launch<TV>(s2, j, nb, bs, dinv, its, spmv);
  PM_HIP(hipEventRecord(j.done, s2));
}

double power_finish(PowerJob& j) {
  double h = 0.0;
  PM_HIP(hipMemcpyAsync(&h, j.nsq, sizeof(double), hipMemcpyDeviceToHost, j.s2));
  PM_HIP(hipStreamSynchronize(j.s2));
  j.release();
  return std::sqrt(h);
}

double estimate_lmax(hipStream_t s, const Sell& A, const double* dinv, int its) {
  return power_lmax(s, A.n, A.bs, dinv, its,
                    [&](hipStream_t ss, const double* v, double* w) { sell_spmv(ss, A, v, w); });
}

// lambda_max(D^-1 A) for a CSR operator (power iteration, fixed start)
// on the CSR arrays directly (lanes per row), without a sliced-ELL copy
// w = A v on the CSR arrays with csr_lanes_for(A) lanes per row
struct CsrSpmv {
  const Csr& A;
  int lanes;
  void operator()(hipStream_t ss, const double* v, double* w) const {
    if (A.bs == 3)
      residual_csr<3, double, false>(ss, A, lanes, A.val, nullptr, v, w);
    else
      residual_csr<1, double, false>(ss, A, lanes, A.val, nullptr, v, w);
  }
};

// the same on the FP32 copy of the values (A.val32)
struct CsrSpmv32 {
  const Csr& A;
  int lanes;
  void operator()(hipStream_t ss, const float* v, float* w) const {
    if (A.bs == 3)
      residual_csr<3, float, false>(ss, A, lanes, A.val32, nullptr, v, w);
    else
      residual_csr<1, float, false>(ss, A, lanes, A.val32, nullptr, v, w);
  }
};

double estimate_lmax_csr(hipStream_t s, const Csr& A, const double* dinv, int its) {
  return power_lmax(s, A.n, A.bs, dinv, its, CsrSpmv{A, csr_lanes_for(A)});
}

void dense_inverse(hipStream_t s, const Csr& A, Hierarchy& H) {
  const int n = A.n * A.bs;
  if (n > 6000) throw Error(PM_EINTERNAL, "AMG: coarsening stalled with " + std::to_string(n) + " unknowns left");
  H.ncoarse = n;
  double* M = dalloc<double>((int64_t)n * 2 * n);
  double* colk = dalloc<double>(n);
  int* status = dalloc<int>(1);
  PM_HIP(hipMemsetAsync(M, 0, sizeof(double) * (size_t)n * 2 * n, s));
  PM_HIP(hipMemsetAsync(status, 0, sizeof(int), s));
  k_dense_from_csr<<<blocks_for(A.n), kBlock, 0, s>>>(A.n, A.bs, A.rowptr, A.col, A.val, M, 2 * n);
  k_set_identity_right<<<blocks_for(n), kBlock, 0, s>>>(n, M);
  PM_CHECK_LAUNCH();
  const int64_t tot = (int64_t)n * 2 * n;
  const size_t lds = sizeof(double) * (size_t)n * n;
  const size_t lds_static = sizeof(double) * (2 * kGjMaxN + 1);
  if (n <= kGjMaxN && lds + lds_static <= (size_t)kGjLdsBytes) {
    // once per process (thread-safe static initialisation)
    static const bool attr_set = [] {
      PM_HIP(hipFuncSetAttribute((const void*)k_gj_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)(kGjLdsBytes - lds_static)));
      return true;
    }();
    (void)attr_set;
    k_gj_lds<<<1, 1024, lds, s>>>(n, M, status);
  } else {
    for (int k = 0; k < n; ++k) {
      k_gj_pivot<<<1, 256, 0, s>>>(n, k, M, colk, status);
      k_gj_elim<<<blocks_for(tot), kBlock, 0, s>>>(n, k, M, colk);
    }
  }
  PM_CHECK_LAUNCH();
  H.coarse_inv = dalloc<double>((int64_t)n * n);
  k_extract_inverse<<<blocks_for((int64_t)n * n), kBlock, 0, s>>>(n, M, H.coarse_inv);
  PM_CHECK_LAUNCH();
  H.cwork = dalloc<double>(2 * (int64_t)n);
  int st = 0;
  PM_HIP(hipMemcpyAsync(&st, status, sizeof(int), hipMemcpyDeviceToHost, s));
  PM_HIP(hipStreamSynchronize(s));
  dfree(M);
  dfree(colk);
  dfree(status);
  if (st) throw Error(PM_EBREAKDOWN, "AMG: coarsest operator is not positive definite");
}

// SG: the structured mesh when A is the finest level of the A_uu (nodes) or
// C~_pi (faces) hierarchy, else nullptr
template <int BS>
void aggregate(hipStream_t s, const Csr& A, double theta, int dist, int* agg, int* nagg_out, uint8_t* strong,
               const Grid* SG) {
  const int n = A.n;
  double* dn = dalloc<double>(n);
  uint8_t* state = dalloc<uint8_t>(n);
  uint64_t* T0 = dalloc<uint64_t>(n);
  uint64_t* T1 = dalloc<uint64_t>(n);
  uint64_t* T2 = dalloc<uint64_t>(n);
  int* und = dalloc<int>(1);
  double* nrm = nullptr;
  BlockNorms<BS> nv{A.val};
  if (BS > 1) {
    nrm = dalloc<double>(A.nnzb);
    k_block_norms<BS><<<blocks_for(A.nnzb), kBlock, 0, s>>>(A.nnzb, A.val, nrm);
    nv.p = nrm;
  }
  with_row_lanes(A, [&](auto g) {
    constexpr int G = decltype(g)::value;
    k_diag_norm<BS, G><<<blocks_for((int64_t)n * G), kBlock, 0, s>>>(n, A.rowptr, A.col, nv, dn);
    k_strength<BS, G><<<blocks_for((int64_t)n * G), kBlock, 0, s>>>(n, A.rowptr, A.col, nv, dn, theta, strong,
                                                                   state);
  });
  PM_CHECK_LAUNCH();
  uint32_t* mask = nullptr;
  if (SG) {
    mask = dalloc<uint32_t>(n);
    PM_HIP(hipMemsetAsync(und, 0, sizeof(int), s));
    if (BS == 3)
      k_mask_nodes<<<blocks_for((int64_t)n * 32), kBlock, 0, s>>>(*SG, A.rowptr, A.col, strong, mask, und);
    else
      k_mask_faces<<<blocks_for(n), kBlock, 0, s>>>(*SG, A.rowptr, A.col, strong, mask, und);
    PM_CHECK_LAUNCH();
    int bad = 0;
    PM_HIP(hipMemcpyAsync(&bad, und, sizeof(int), hipMemcpyDeviceToHost, s));
    PM_HIP(hipStreamSynchronize(s));
    if (bad) {  // a strong column outside the stencil: use the CSR rounds
      dfree(mask);
      mask = nullptr;
    }
  }
  auto mis_pass = [&](const uint64_t* Tin, uint64_t* Tout, const int* go) {
    if (!mask)
      launch_mis_max(s, A, strong, Tin, Tout, go);
    else if (BS == 3)
      k_mis_max_nodes<<<blocks_for(n), kBlock, 0, s>>>(*SG, mask, Tin, Tout, go);
    else
      k_mis_max_faces<<<blocks_for(n), kBlock, 0, s>>>(*SG, mask, Tin, Tout, go);
  };
  // round r runs if round r-1 left undecided rows (flag[(r+1)&1]) and sets
  // flag[r&1]; the host looks every kRoundsPerCheck rounds
  constexpr int kRoundsPerCheck = 5;
  int* flag = dalloc<int>(2);
  PM_HIP(hipMemsetD32Async((hipDeviceptr_t)flag, 1, 2, s));
  for (int round = 0;; ++round) {
    int* cur = flag + (round & 1);
    const int* prev = flag + ((round + 1) & 1);
    PM_HIP(hipMemsetAsync(cur, 0, sizeof(int), s));
    k_mis_init<<<blocks_for(n), kBlock, 0, s>>>(n, state, 0x12345u, T0, prev);
    mis_pass(T0, T1, prev);
    if (dist == 2) mis_pass(T1, T2, prev);
    k_mis_update<<<blocks_for(n), kBlock, 0, s>>>(n, T0, dist == 2 ? T2 : T1, state, cur, prev);
    PM_CHECK_LAUNCH();
    if ((round + 1) % kRoundsPerCheck == 0) {
      int h = 0;
      PM_HIP(hipMemcpyAsync(&h, cur, sizeof(int), hipMemcpyDeviceToHost, s));
      PM_HIP(hipStreamSynchronize(s));
      if (h == 0) break;
      if (round >= 999) {
        dfree(flag);
        throw Error(PM_EINTERNAL, "AMG: independent-set rounds did not terminate");
      }
    }
  }
  dfree(flag);
  int* flags = dalloc<int>(n);
  int* root_id = dalloc<int>(n + 1);
  k_root_flags<<<blocks_for(n), kBlock, 0, s>>>(n, state, flags);
  int nagg = 0;
  exclusive_scan(s, flags, root_id, n, &nagg);
  int* agg1 = dalloc<int>(n);
  PM_HIP(hipMemsetAsync(und, 0, sizeof(int), s));
  with_row_lanes(A, [&](auto g) {
    constexpr int G = decltype(g)::value;
    k_agg_phase1<BS, G><<<blocks_for((int64_t)n * G), kBlock, 0, s>>>(n, A.rowptr, A.col, nv, strong, state,
                                                                     root_id, agg1);
    k_agg_phase2<BS, G><<<blocks_for((int64_t)n * G), kBlock, 0, s>>>(n, A.rowptr, A.col, nv, strong, agg1, agg,
                                                                     und);
  });
  PM_CHECK_LAUNCH();
  int st = 0;
  PM_HIP(hipMemcpyAsync(&st, und, sizeof(int), hipMemcpyDeviceToHost, s));
  PM_HIP(hipStreamSynchronize(s));
  for (void* p : {(void*)dn, (void*)state, (void*)T0, (void*)T1, (void*)T2, (void*)und,
                  (void*)flags, (void*)root_id, (void*)agg1, (void*)mask, (void*)nrm})
    dfree(p);
  if (st) throw Error(PM_EINTERNAL, "AMG: aggregation left a connected node unassigned");
  *nagg_out = nagg;
}

// ---------------------------------------------------------------------------
// Rigid-body near kernel for the A_uu hierarchy (the analogue of the paper's
// M_III^(h) preconditioner, Sec. 5).  Every coarse "node" is an aggregate J
// with a centroid c_J and six unknowns: a translation T_J and a rotation
// Omega_J (two 3x3 block rows, 2J and 2J+1).  The tentative prolongator
// interpolates rigid motions exactly:
//   finest level, node i of J:        u_i = T_J + Omega_J x (x_i - c_J)
//   coarser level, aggregate I of J:  T_I = T_J + Omega_J x (c_I - c_J),
//                                     Omega_I = Omega_J
// i.e. block rows [I | rot(d)] (and [0 | I]), rot(d) w = w x d, so the
// translations and rotations of every level are those of the finest.  The
// coarse levels are aggregated on the graph of the aggregate pairs.  A
// rotation that an aggregate cannot carry (one node, or nodes on a line
// through the centroid along the axis) gives a zero prolongator column; the
// coarse operator's zero diagonal entries there are set to one.  One thread
// per aggregate takes its members in increasing order (deterministic).
__global__ void k_agg_count(int n, const int* __restrict__ agg, int* __restrict__ cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && agg[i] >= 0) atomicAdd(&cnt[agg[i]], 1);
}

__global__ void k_agg_fill(int n, const int* __restrict__ agg, const int* __restrict__ aoff, int* __restrict__ cur,
                           int* __restrict__ list) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || agg[i] < 0) return;
  const int J = agg[i];
  list[aoff[J] + atomicAdd(&cur[J], 1)] = i;
}

// blocks per row of the tentative prolongator: finest level 2 (translation
// and rotation columns of the node's aggregate); paired levels 2 for the
// translation row of an aggregated member, 1 for its rotation row
__global__ void k_rbm_count(int n, const int* __restrict__ agg, int paired, int* __restrict__ f) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int m = paired ? i >> 1 : i;
  f[i] = agg[m] < 0 ? 0 : ((paired && (i & 1)) ? 1 : 2);
}

// rot(d): column a is e_a x d
__device__ inline void rot_block(const double d[3], double S[9]) {
  S[0] = 0.0;   S[1] = d[2];  S[2] = -d[1];
  S[3] = -d[2]; S[4] = 0.0;   S[5] = d[0];
  S[6] = d[1];  S[7] = -d[0]; S[8] = 0.0;
}

__global__ void k_rbm_ptent(int nagg, const int* __restrict__ aoff, int* __restrict__ list,
                            const double* __restrict__ pos, int paired, const int* __restrict__ prow,
                            int* __restrict__ pcol, double* __restrict__ pval, double* __restrict__ cen) {
  const int J = blockIdx.x * blockDim.x + threadIdx.x;
  if (J >= nagg) return;
  const int b = aoff[J], e = aoff[J + 1], m = e - b;
  for (int p = b + 1; p < e; ++p) {  // the members in increasing order
    const int v = list[p];
    int q = p - 1;
    while (q >= b && list[q] > v) {
      list[q + 1] = list[q];
      --q;
    }
    list[q + 1] = v;
  }
  double c[3] = {0.0, 0.0, 0.0};
  for (int p = b; p < e; ++p)
    for (int a = 0; a < 3; ++a) c[a] += pos[3 * (size_t)list[p] + a];
  for (int a = 0; a < 3; ++a) {
    c[a] /= (double)m;
    cen[3 * (size_t)J + a] = c[a];
  }
  for (int p = b; p < e; ++p) {
    const int i = list[p];
    double d[3], S[9];
    for (int a = 0; a < 3; ++a) d[a] = pos[3 * (size_t)i + a] - c[a];
    rot_block(d, S);
    const int r0 = paired ? 2 * i : i;  // the (translation) block row of the member
    const int e0 = prow[r0];
    pcol[e0] = 2 * J;
    pcol[e0 + 1] = 2 * J + 1;
    for (int q = 0; q < 9; ++q) {
      pval[(size_t)e0 * 9 + q] = (q % 4 == 0) ? 1.0 : 0.0;
      pval[(size_t)(e0 + 1) * 9 + q] = S[q];
    }
    if (paired) {  // the rotation row: Omega_I = Omega_J
      const int e1 = prow[r0 + 1];
      pcol[e1] = 2 * J + 1;
      for (int q = 0; q < 9; ++q) pval[(size_t)e1 * 9 + q] = (q % 4 == 0) ? 1.0 : 0.0;
    }
  }
}

// Graph of the aggregate pairs of a paired level: super-row I merges block
// rows 2I and 2I+1 (columns J = col / 2, both lists sorted), with the value
// sqrt(sum of the squared Frobenius norms of the blocks it covers)
__global__ void k_pair_count(int n2, const int* __restrict__ rp, const int* __restrict__ col,
                             int* __restrict__ cnt) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= n2) return;
  int a = rp[2 * I], b = rp[2 * I + 1];
  const int ae = rp[2 * I + 1], be = rp[2 * I + 2];
  int k = 0, last = -1;
  while (a < ae || b < be) {
    const int ja = a < ae ? col[a] >> 1 : INT_MAX, jb = b < be ? col[b] >> 1 : INT_MAX;
    const int j = min(ja, jb);
    if (j == ja) ++a; else ++b;
    if (j != last) {
      ++k;
      last = j;
    }
  }
  cnt[I] = k;
}

__global__ void k_pair_fill(int n2, const int* __restrict__ rp, const int* __restrict__ col,
                            const double* __restrict__ val, const int* __restrict__ srp, int* __restrict__ scol,
                            double* __restrict__ sval) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= n2) return;
  int a = rp[2 * I], b = rp[2 * I + 1];
  const int ae = rp[2 * I + 1], be = rp[2 * I + 2];
  int k = srp[I] - 1, last = -1;
  double acc = 0.0;
  while (a < ae || b < be) {
    const int ja = a < ae ? col[a] >> 1 : INT_MAX, jb = b < be ? col[b] >> 1 : INT_MAX;
    const int j = min(ja, jb);
    const int eb = (j == ja) ? a++ : b++;
    if (j != last) {
      if (last >= 0) sval[k] = sqrt(acc);
      ++k;
      scol[k] = j;
      acc = 0.0;
      last = j;
    }
    for (int q = 0; q < 9; ++q) acc += val[(size_t)eb * 9 + q] * val[(size_t)eb * 9 + q];
  }
  if (last >= 0) sval[k] = sqrt(acc);
}

// tentative prolongator of a rigid-body level; cen receives the aggregates'
// centroids (nagg x 3, the positions of the next level)
void build_rbm_ptent(hipStream_t s, int nb, int nmem, const int* agg, int nagg, const double* pos, bool paired,
                     Csr& Pt, double* cen) {
  int* cnt = dalloc<int>(nagg);
  int* aoff = dalloc<int>(nagg + 1);
  int* list = dalloc<int>(std::max(nmem, 1));
  PM_HIP(hipMemsetAsync(cnt, 0, sizeof(int) * (size_t)nagg, s));
  k_agg_count<<<blocks_for(nmem), kBlock, 0, s>>>(nmem, agg, cnt);
  PM_CHECK_LAUNCH();
  int total = 0;
  exclusive_scan(s, cnt, aoff, nagg, &total);
  PM_HIP(hipMemsetAsync(cnt, 0, sizeof(int) * (size_t)nagg, s));
  k_agg_fill<<<blocks_for(nmem), kBlock, 0, s>>>(nmem, agg, aoff, cnt, list);
  PM_CHECK_LAUNCH();
  dfree(cnt);
  Pt.bs = 3;
  Pt.n = nb;
  Pt.m = 2 * nagg;
  Pt.rowptr = dalloc<int>(nb + 1);
  int* f = dalloc<int>(nb);
  k_rbm_count<<<blocks_for(nb), kBlock, 0, s>>>(nb, agg, paired ? 1 : 0, f);
  PM_CHECK_LAUNCH();
  int nnz = 0;
  exclusive_scan(s, f, Pt.rowptr, nb, &nnz);
  dfree(f);
  Pt.nnzb = nnz;
  Pt.col = dalloc<int>(nnz);
  Pt.val = dalloc<double>((int64_t)nnz * 9);
  k_rbm_ptent<<<blocks_for(nagg), kBlock, 0, s>>>(nagg, aoff, list, pos, paired ? 1 : 0, Pt.rowptr, Pt.col,
                                                   Pt.val, cen);
  PM_CHECK_LAUNCH();
  dfree(aoff);
  dfree(list);
}

// P = P_tent - omega D^-1 (A P_tent) on the pattern of A P_tent, for a
// general P_tent (whose pattern is contained in that of A P_tent)
template <int BS>
__global__ void k_smooth_p_gen(int n, const double* __restrict__ dinv, double omega, const int* __restrict__ rp,
                               const int* __restrict__ col, double* __restrict__ val, const int* __restrict__ trp,
                               const int* __restrict__ tcol, const double* __restrict__ tval) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double* D = dinv + (size_t)i * BS * BS;
  int f = trp[i];
  const int f1 = trp[i + 1];
  for (int e = rp[i]; e < rp[i + 1]; ++e) {
    double* v = val + (size_t)e * BS * BS;
    const bool hit = f < f1 && tcol[f] == col[e];  // both rows sorted by column
    double o[BS * BS];
    for (int a = 0; a < BS; ++a)
      for (int b = 0; b < BS; ++b) {
        double sum = 0.0;
        for (int t = 0; t < BS; ++t) sum += D[a * BS + t] * v[t * BS + b];
        o[a * BS + b] = -omega * sum + (hit ? tval[(size_t)f * BS * BS + a * BS + b] : 0.0);
      }
    for (int q = 0; q < BS * BS; ++q) v[q] = o[q];
    if (hit) ++f;
  }
}

// diagonal entries that are exactly zero (coarse unknowns of dropped
// near-kernel columns: zero row and column) set to one
template <int BS>
__global__ void k_fix_zero_diag(int n, const int* __restrict__ rp, const int* __restrict__ col,
                                double* __restrict__ val) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int e = rp[i]; e < rp[i + 1]; ++e)
    if (col[e] == i)
      for (int a = 0; a < BS; ++a) {
        double& d = val[(size_t)e * BS * BS + a * BS + a];
        if (d == 0.0) d = 1.0;
      }
}

// lmax_job: the level's own power iteration when it is still running on the
// side stream (taken here if the transfer needs it).
// pos: positions of the level's nodes (rigid-body hierarchies: the finest
// node coordinates, then the aggregate centroids of the paired levels, whose
// block rows come in translation/rotation pairs); *cen_next receives the
// next level's (device, owned by the caller)
template <int BS>
void build_level_transfer(hipStream_t s, Level& L, const AmgParams& prm, Csr& Acoarse, const Grid* SG,
                          PowerJob* lmax_job, const double* pos, bool paired, double** cen_next) {
  const Csr& A = L.A;
  const int n = A.n;
  const bool rbm = BS == 3 && pos != nullptr;
  uint8_t* strong = dalloc<uint8_t>(A.nnzb);
  int nagg = 0;
  const int nmem = paired ? n / 2 : n;  // aggregated units: nodes, or aggregate pairs
  int* agg = dalloc<int>(nmem);
  if (paired) {
    // aggregation on the graph of the pairs; A itself is not filtered
    Csr Sg;
    Sg.bs = 1;
    Sg.n = Sg.m = nmem;
    Sg.rowptr = dalloc<int>(nmem + 1);
    int* cnt = dalloc<int>(nmem);
    k_pair_count<<<blocks_for(nmem), kBlock, 0, s>>>(nmem, A.rowptr, A.col, cnt);
    PM_CHECK_LAUNCH();
    int snnz = 0;
    exclusive_scan(s, cnt, Sg.rowptr, nmem, &snnz);
    dfree(cnt);
    Sg.nnzb = snnz;
    Sg.col = dalloc<int>(snnz);
    Sg.val = dalloc<double>(snnz);
    k_pair_fill<<<blocks_for(nmem), kBlock, 0, s>>>(nmem, A.rowptr, A.col, A.val, Sg.rowptr, Sg.col, Sg.val);
    PM_CHECK_LAUNCH();
    uint8_t* sstrong = dalloc<uint8_t>(snnz);
    aggregate<1>(s, Sg, prm.theta, prm.agg_dist, agg, &nagg, sstrong, nullptr);
    dfree(sstrong);
    Sg.free_all();
    PM_HIP(hipMemsetAsync(strong, 1, (size_t)A.nnzb, s));
  } else {
    aggregate<BS>(s, A, prm.theta, prm.agg_dist, agg, &nagg, strong, SG);
  }
  if (nagg == 0) {
    // every row isolated (no strong coupling): no coarser level; the caller
    // makes this level the coarsest
    dfree(agg);
    dfree(strong);
    if (lmax_job && lmax_job->pending()) L.lmax = power_finish(*lmax_job);
    Acoarse.free_all();
    Acoarse = Csr();
    return;
  }
  // tentative prolongator
  Csr Pt;
  int* f = dalloc<int>(n);
  if (rbm) {
    *cen_next = dalloc<double>(3 * (int64_t)std::max(nagg, 1));
    build_rbm_ptent(s, n, nmem, agg, nagg, pos, paired, Pt, *cen_next);
  } else {
    Pt.bs = BS;
    Pt.n = n;
    Pt.m = nagg;
    k_count_aggregated<<<blocks_for(n), kBlock, 0, s>>>(n, agg, f);
    Pt.rowptr = dalloc<int>(n + 1);
    int nnz = 0;
    exclusive_scan(s, f, Pt.rowptr, n, &nnz);
    Pt.nnzb = nnz;
    Pt.col = dalloc<int>(nnz);
    Pt.val = dalloc<double>((int64_t)nnz * BS * BS);
    k_ptent<BS><<<blocks_for(n), kBlock, 0, s>>>(n, agg, Pt.rowptr, Pt.col, Pt.val);
    PM_CHECK_LAUNCH();
  }
  const int* pt_agg = rbm ? nullptr : agg;  // the tentative-product fast path needs one identity block per row
  // filtered operator A_F (strong couplings, weak ones lumped on the diagonal);
  // when no nonzero coupling is weak A_F = A and the level's D^-1, lmax serve
  Csr AF;
  AF.bs = BS;
  AF.n = AF.m = n;
  int* weak_rows = dalloc<int>(1);
  PM_HIP(hipMemsetAsync(weak_rows, 0, sizeof(int), s));
  with_row_lanes(A, [&](auto g) {
    constexpr int G = decltype(g)::value;
    k_filter_count<G><<<blocks_for((int64_t)n * G), kBlock, 0, s>>>(n, A.rowptr, A.col, strong, f, weak_rows);
  });
  AF.rowptr = dalloc<int>(n + 1);
  int fnnz = 0;
  exclusive_scan(s, f, AF.rowptr, n, &fnnz);
  dfree(f);
  int nweak = 0;
  PM_HIP(hipMemcpyAsync(&nweak, weak_rows, sizeof(int), hipMemcpyDeviceToHost, s));
  PM_HIP(hipStreamSynchronize(s));
  dfree(weak_rows);
  const bool filtered = nweak > 0;
  double* dinvF = nullptr;
  double lF = 0.0;
  Csr P;
  if (filtered) {
    AF.nnzb = fnnz;
    AF.col = dalloc<int>(fnnz);
    AF.val = dalloc<double>((int64_t)fnnz * BS * BS);
    with_row_lanes(A, [&](auto g) {
      constexpr int G = decltype(g)::value;
      k_filter_fill<BS, G><<<blocks_for((int64_t)n * G), kBlock, 0, s>>>(n, A.rowptr, A.col, A.val, strong,
                                                                         AF.rowptr, AF.col, AF.val);
    });
    PM_CHECK_LAUNCH();
    dinvF = dalloc<double>((int64_t)n * BS * BS);
    block_diag_inverse(s, AF, dinvF);
    // smoothed prolongator P = (I - 4/(3 lmax) D_F^-1 A_F) P_tent on the pattern of A_F P_tent;
    // lambda_max(D_F^-1 A_F) on the side stream, if any, during the product
    // (in mixed precision on an FP32 copy of A_F, as the V-cycles apply theirs)
    const int lanesF = csr_lanes_for(AF);
    if (prm.fp32) {
      const int64_t nv = AF.nnzb * BS * BS;
      AF.val32 = dalloc<float>(nv);
      k_to_float<<<blocks_for(nv), kBlock, 0, s>>>(nv, AF.val, AF.val32);
      PM_CHECK_LAUNCH();
    }
    if (prm.side) {
      PowerJob jf;
      if (prm.fp32)
        power_start<float>(jf, s, prm.side, n, BS, dinvF, prm.power_its, CsrSpmv32{AF, lanesF});
      else
        power_start(jf, s, prm.side, n, BS, dinvF, prm.power_its, CsrSpmv{AF, lanesF});
      spgemm(s, AF, Pt, P, pt_agg);
      lF = power_finish(jf);
    } else {
      lF = prm.fp32 ? power_lmax<float>(s, n, BS, dinvF, prm.power_its, CsrSpmv32{AF, lanesF})
                    : estimate_lmax_csr(s, AF, dinvF, prm.power_its);
      spgemm(s, AF, Pt, P, pt_agg);
    }
  } else {
    spgemm(s, A, Pt, P, pt_agg);
    if (lmax_job && lmax_job->pending()) L.lmax = power_finish(*lmax_job);
    lF = L.lmax;
  }
  dfree(strong);
  AF.free_all();
  const double omega = 4.0 / (3.0 * lF);
  if (rbm)
    k_smooth_p_gen<BS><<<blocks_for(n), kBlock, 0, s>>>(n, filtered ? dinvF : L.dinv, omega, P.rowptr, P.col,
                                                        P.val, Pt.rowptr, Pt.col, Pt.val);
  else
    k_smooth_p<BS><<<blocks_for(n), kBlock, 0, s>>>(n, agg, filtered ? dinvF : L.dinv, omega, P.rowptr, P.col,
                                                    P.val);
  PM_CHECK_LAUNCH();
  Pt.free_all();
  if (prm.p_trunc > 0.0) truncate_p<BS>(s, P, prm.p_trunc, rbm);
  dfree(dinvF);
  dfree(agg);
  // Galerkin coarse operator
  Csr AP, R;
  spgemm(s, A, P, AP);
  csr_transpose(s, P, R);
  spgemm(s, R, AP, Acoarse);
  AP.free_all();
  if (rbm) {
    k_fix_zero_diag<BS><<<blocks_for(Acoarse.n), kBlock, 0, s>>>(Acoarse.n, Acoarse.rowptr, Acoarse.col,
                                                                 Acoarse.val);
    PM_CHECK_LAUNCH();
  }
  csr_to_sell(s, P, L.P, prm.fp32);
  L.R = R;
  if (prm.fp32) {
    const int64_t nv = R.nnzb * BS * BS;
    L.R.val32 = dalloc<float>(nv);
    k_to_float<<<blocks_for(nv), kBlock, 0, s>>>(nv, R.val, L.R.val32);
    PM_CHECK_LAUNCH();
  }
  P.free_all();
}

void alloc_level_vectors(Level& L, bool fp32) {
  const int64_t m = (int64_t)L.n * L.bs;
  L.x = dalloc<double>(m);
  L.b = dalloc<double>(m);
  L.r = dalloc<double>(m);
  L.d = dalloc<double>(m);
  L.t = dalloc<double>(m);
  if (fp32) {
    L.xf = dalloc<float>(m);
    L.bf = dalloc<float>(m);
    L.rf = dalloc<float>(m);
    L.df = dalloc<float>(m);
    L.tf = dalloc<float>(m);
  }
}

// Chebyshev smoothing of A x = b on level L, x0 = 0 if zero_init.
// Returns the buffer holding the result (x or t).
template <int BS, class T>
T* chebyshev(hipStream_t s, const Level& L, const AmgParams& prm, const T* b, T* x, T* t, T* d, bool zero_init,
             const T* val, const T* dinv, int prof_id, const LatticeOp* lat, const CellPiOp* cpi, const Grid& G) {
  const double lo = prm.cheb_lower * L.lmax, hi = prm.cheb_upper * L.lmax;
  const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo);
  const double sigma = theta / delta;
  double rho = 1.0 / sigma;
  const int n = L.n;
  const int nth = L.As.nslices * kSlice;
  T* cur = x;
  T* nxt = t;
  int k0 = 0;
  // from zero, start in t: pre-smoothing then ends in x (even degree) or t
  // (odd), and the post-smoothing steps that follow end in x either way
  if (zero_init) std::swap(cur, nxt);
  if (zero_init) {
    k_cheb_first<BS, T><<<blocks_for(n), kBlock, 0, s>>>(n, dinv, b, (T)(1.0 / theta), cur, d);
    k0 = 1;
  }
  for (int k = k0; k < prm.cheb_degree; ++k) {
    double c1, c2;
    if (k == 0) {
      c1 = 0.0;
      c2 = 1.0 / theta;
    } else {
      const double rn = 1.0 / (2.0 * sigma - rho);
      c1 = rn * rho;
      c2 = 2.0 * rn / delta;
      rho = rn;
    }
    g_prof.begin(s, prof_id);
    if (L.csr_cycle) {
      cheb_step_csr<BS, T>(s, L, val, dinv, b, cur, nxt, d, (T)c1, (T)c2);
      g_prof.end(s, prof_id, 0.0);
    } else if (BS == 1 && cpi) {
      cellpi_cheb_step<T>(s, G, *cpi, dinv, b, cur, nxt, d, (T)c1, (T)c2);
      // algorithmic bytes: 21 packed values per cell; x/b/d read, x/d written, D^-1 per face
      g_prof.end(s, prof_id, (double)G.nc * 21 * sizeof(T) + (double)n * sizeof(T) * 6);
    } else if (BS == 3 && lat) {
      lattice_cheb_step<T>(s, G, *lat, dinv, b, cur, nxt, d, (T)c1, (T)c2);
      // algorithmic bytes: x/b/d read, x/d written, D^-1 blocks, cell moduli;
      // flops: 576 stencil multiply-adds per node
      g_prof.end(s, prof_id, (double)n * BS * sizeof(T) * 5 + (double)n * BS * BS * sizeof(T) +
                                 (double)G.nc * sizeof(T), 2.0 * 576 * (double)n);
    } else {
      k_cheb_step<BS, T><<<blocks_for(nth), kBlock, 0, s>>>(n, L.As.sptr, L.As.perm, L.As.col, val, dinv, b, cur, nxt, d,
                                                            (T)c1, (T)c2);
      // algorithmic bytes: blocks + column ids, x/b/d read, x/d written, D^-1 blocks
      g_prof.end(s, prof_id,
                 (double)L.As.nnzb * (BS * BS * sizeof(T) + 4) + (double)n * BS * sizeof(T) * 5 +
                     (double)n * BS * BS * sizeof(T));
    }
    T* tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
  return cur;
}

template <int BS, class T>
void vcycle_level(hipStream_t s, Hierarchy& H, const AmgParams& prm, int l, const T* b, T* x);

template <int BS, class T>
struct LevelPtrs;
template <int BS>
struct LevelPtrs<BS, double> {
  static double* X(Level& L) { return L.x; }
  static double* B(Level& L) { return L.b; }
  static double* Rr(Level& L) { return L.r; }
  static double* D(Level& L) { return L.d; }
  static double* Tt(Level& L) { return L.t; }
  static const double* AV(const Sell& S) { return S.val; }
  static const double* CV(const Csr& S) { return S.val; }
  static const double* DI(const Level& L) { return L.dinv; }
};
template <int BS>
struct LevelPtrs<BS, float> {
  static float* X(Level& L) { return L.xf; }
  static float* B(Level& L) { return L.bf; }
  static float* Rr(Level& L) { return L.rf; }
  static float* D(Level& L) { return L.df; }
  static float* Tt(Level& L) { return L.tf; }
  static const float* AV(const Sell& S) { return S.val32; }
  static const float* CV(const Csr& S) { return S.val32; }
  static const float* DI(const Level& L) { return L.dinv32; }
};

template <int BS, class T>
void vcycle_level(hipStream_t s, Hierarchy& H, const AmgParams& prm, int l, const T* b, T* x) {
  using LP = LevelPtrs<BS, T>;
  Level& L = H.L[l];
  const int n = L.n;
  if (l == (int)H.L.size() - 1) {
    k_dense_gemv<T><<<(H.ncoarse + 3) / 4, 256, 0, s>>>(H.ncoarse, H.coarse_inv, b, x);
    PM_CHECK_LAUNCH();
    return;
  }
  const T* AV = L.csr_cycle ? LP::CV(L.A) : LP::AV(L.As);
  const T* DI = LP::DI(L);
  T* d = LP::D(L);
  T* t = LP::Tt(L);
  T* r = LP::Rr(L);
  // pre-smoothing from zero
  const int prof_id = l == 0 ? (BS == 3 ? kProfChebU0 : kProfChebPi0) : 0;
  const LatticeOp* lat = (l == 0 && BS == 3) ? H.lat : nullptr;
  const CellPiOp* cpi = (l == 0 && BS == 1) ? H.cpi : nullptr;
  T* cur = chebyshev<BS, T>(s, L, prm, b, x, t, d, true, AV, DI, prof_id, lat, cpi, H.grid);
  // residual, restriction
  if (lat) {
    g_prof.begin(s, kProfResidU0);
    lattice_residual<T>(s, H.grid, *lat, b, cur, r);
    // algorithmic bytes: x, b read, r written, cell moduli; flops: 576 per node
    g_prof.end(s, kProfResidU0, (double)n * BS * sizeof(T) * 3 + (double)H.grid.nc * sizeof(T), 2.0 * 576 * (double)n);
  } else if (cpi) {
    g_prof.begin(s, kProfResidPi0);
    cellpi_residual<T>(s, H.grid, *cpi, b, cur, r);
    // algorithmic bytes: x, b read, r written, the per-cell element matrices
    g_prof.end(s, kProfResidPi0, (double)n * sizeof(T) * 3 + (double)H.grid.nc * cpi->nvals * sizeof(T));
  } else if (L.csr_cycle) {
    residual_csr<BS, T, true>(s, L.A, L.csr_lanes, AV, b, cur, r);
  } else {
    const int nth = L.As.nslices * kSlice;
    k_residual<BS, T><<<blocks_for(nth), kBlock, 0, s>>>(n, L.As.sptr, L.As.perm, L.As.col, AV, b, cur, r);
  }
  Level& C = H.L[l + 1];
  const int rprof = l == 0 ? (BS == 3 ? kProfRestrictU0 : kProfRestrictPi0) : 0;
  g_prof.begin(s, rprof);
  residual_csr<BS, T, false>(s, L.R, restrict_lanes_for(L.R), LP::CV(L.R), nullptr, r, LP::B(C));
  g_prof.end(s, rprof, (double)L.R.nnzb * (BS * BS * sizeof(T) + 4) + (double)(n + C.n) * BS * sizeof(T));
  vcycle_level<BS, T>(s, H, prm, l + 1, LP::B(C), LP::X(C));
  const int pth = L.P.nslices * kSlice;
  const int pprof = l == 0 ? (BS == 3 ? kProfProlongU0 : kProfProlongPi0) : 0;
  g_prof.begin(s, pprof);
  k_sell_apply<BS, T, true><<<blocks_for(pth), kBlock, 0, s>>>(L.P.n, L.P.sptr, L.P.perm, L.P.col, LP::AV(L.P),
                                                                LP::X(C), cur);
  // algorithmic bytes: P blocks and column ids, coarse x read, fine x read and written
  g_prof.end(s, pprof, (double)L.P.nnzb * (BS * BS * sizeof(T) + 4) + (double)C.n * BS * sizeof(T) +
                           2.0 * n * BS * sizeof(T));
  PM_CHECK_LAUNCH();
  // post-smoothing from the corrected iterate
  T* other = (cur == x) ? t : x;
  T* res = chebyshev<BS, T>(s, L, prm, b, cur, other, d, false, AV, DI, prof_id, lat, cpi, H.grid);
  if (res != x) PM_HIP(hipMemcpyAsync(x, res, sizeof(T) * (size_t)n * BS, hipMemcpyDeviceToDevice, s));
}

}  // namespace

void amg_setup(hipStream_t s, const Csr& A0, const AmgParams& prm, Hierarchy& H, const LatticeOp* lat,
               const Grid* G, const CellPiOp* cpi) {
  H.free_all();
  H.bs = A0.bs;
  H.lat = (lat && lat->on && G && A0.bs == 3) ? lat : nullptr;
  H.cpi = (cpi && cpi->on && G && A0.bs == 1) ? cpi : nullptr;
  if (H.lat || H.cpi) H.grid = *G;
  H.fp32 = prm.fp32;
  H.prm = prm;
  double nnz_total = 0.0, nnz0 = (double)A0.nnzb;
  const char* env = getenv("PM_AMG_VERBOSE");
  const bool verbose = env && env[0] == '1';
  // level 0 refers to the caller's operator (which outlives the hierarchy:
  // both are rebuilt together); coarser levels are owned
  Csr cur = A0;
  cur.val32 = nullptr;
  cur.borrowed = true;
  // rigid-body near kernel: positions of the current level's nodes
  const double* rbm_pos = (prm.rbm && prm.coords && H.bs == 3 && G && A0.n == G->nn) ? prm.coords : nullptr;
  bool rbm_paired = false;
  double* rbm_cen = nullptr;  // owned centroids of the current paired level
  struct CenGuard {
    double*& p;
    ~CenGuard() { dfree(p); }
  } cen_guard{rbm_cen};
  for (int l = 0;; ++l) {
    H.L.emplace_back();
    Level& L = H.L.back();
    L.bs = cur.bs;
    L.n = cur.n;
    L.A = cur;
    cur = Csr();
    nnz_total += (double)L.A.nnzb;
    const bool last = (L.n <= prm.coarse_max) || (l + 1 >= prm.max_levels);
    alloc_level_vectors(L, prm.fp32);
    const bool on_lattice = (l == 0 && (H.lat || H.cpi));
    // long rows on a small level: latency-bound with one thread per row
    // small coarse levels with long rows: CSR with lanes per row (one thread
    // per sliced-ELL row is latency-bound there); large levels keep sliced ELL
    L.csr_cycle = !last && l > 0 && L.n <= 262144 && (double)L.A.nnzb >= 12.0 * L.n;
    L.csr_lanes = csr_lanes_for(L.A);
    if (L.csr_cycle) {
      if (prm.fp32) {
        const int64_t nv = L.A.nnzb * L.bs * L.bs;
        L.A.val32 = dalloc<float>(nv);
        k_to_float<<<blocks_for(nv), kBlock, 0, s>>>(nv, L.A.val, L.A.val32);
        PM_CHECK_LAUNCH();
      }
    } else if (!on_lattice) {
      csr_to_sell(s, L.A, L.As, prm.fp32);
    }
    if (last) {
      dense_inverse(s, L.A, H);
      break;
    }
    L.dinv = dalloc<double>((int64_t)L.n * L.bs * L.bs);
    block_diag_inverse(s, L.A, L.dinv);
    if (prm.fp32) {
      L.dinv32 = dalloc<float>((int64_t)L.n * L.bs * L.bs);
      k_to_float<<<blocks_for((int64_t)L.n * L.bs * L.bs), kBlock, 0, s>>>((int64_t)L.n * L.bs * L.bs, L.dinv,
                                                                         L.dinv32);
      PM_CHECK_LAUNCH();
    }
    // the finest level's lambda_max runs on the side stream, if any, during
    // the aggregation (the transfer takes it when it needs it).  In mixed
    // precision every level's iteration runs on the FP32 operator and D^-1
    // that its V-cycle applies.
    PowerJob job;
    if (on_lattice && prm.fp32) {
      auto op = [&](hipStream_t ss, const float* v, float* w) {
        if (H.lat)
          lattice_apply(ss, H.grid, *H.lat, v, w);
        else
          cellpi_apply(ss, H.grid, *H.cpi, v, w);
      };
      if (prm.side)
        power_start<float>(job, s, prm.side, L.n, L.bs, L.dinv32, prm.power_its, op);
      else
        L.lmax = power_lmax<float>(s, L.n, L.bs, L.dinv32, prm.power_its, op);
    } else if (on_lattice) {
      auto op = [&](hipStream_t ss, const double* v, double* w) {
        if (H.lat)
          lattice_apply(ss, H.grid, *H.lat, v, w);
        else
          cellpi_apply(ss, H.grid, *H.cpi, v, w);
      };
      if (prm.side)
        power_start(job, s, prm.side, L.n, L.bs, L.dinv, prm.power_its, op);
      else
        L.lmax = power_lmax(s, L.n, L.bs, L.dinv, prm.power_its, op);
    } else if (L.csr_cycle && prm.fp32) {
      L.lmax = power_lmax<float>(s, L.n, L.bs, L.dinv32, prm.power_its, CsrSpmv32{L.A, L.csr_lanes});
    } else if (prm.fp32) {
      const Sell& As = L.As;
      L.lmax = power_lmax<float>(s, L.n, L.bs, L.dinv32, prm.power_its,
                                 [&](hipStream_t ss, const float* v, float* w) { sell_spmv32(ss, As, v, w); });
    } else if (L.csr_cycle) {
      const Csr& A = L.A;
      L.lmax = power_lmax(s, L.n, L.bs, L.dinv, prm.power_its, [&](hipStream_t ss, const double* v, double* w) {
        if (L.bs == 3)
          residual_csr<3, double, false>(ss, A, L.csr_lanes, A.val, nullptr, v, w);
        else
          residual_csr<1, double, false>(ss, A, L.csr_lanes, A.val, nullptr, v, w);
      });
    } else
      L.lmax = estimate_lmax(s, L.As, L.dinv, prm.power_its);
    auto report = [&] {
      if (verbose)
        fprintf(stderr,
                "[amg bs=%d] level %d: rows %d, blocks %lld (%.1f/row), lmax(D^-1 A) %.4f, sliced-ELL fill %.3f\n",
                L.bs, l, L.n, (long long)L.A.nnzb, (double)L.A.nnzb / std::max(1, L.n), L.lmax,
                L.As.nslices ? (double)L.As.ncols * kSlice / std::max<int64_t>(1, L.A.nnzb) : 0.0);
    };
    if (!job.pending()) report();
    Csr Ac;
    const auto tl0 = std::chrono::steady_clock::now();
    // the finest level of either hierarchy is the structured node or face graph
    const Grid* sg =
        (l == 0 && G && ((L.bs == 3 && L.n == G->nn) || (L.bs == 1 && L.n == G->nf))) ? G : nullptr;
    double* cen_next = nullptr;
    if (L.bs == 3)
      build_level_transfer<3>(s, L, prm, Ac, sg, &job, rbm_pos, rbm_paired, &cen_next);
    else
      build_level_transfer<1>(s, L, prm, Ac, sg, &job, nullptr, false, &cen_next);
    if (cen_next) {
      dfree(rbm_cen);
      rbm_cen = cen_next;
      rbm_pos = cen_next;
      rbm_paired = true;
    }
    if (job.pending()) {
      L.lmax = power_finish(job);
      report();
    }
    if (verbose) {
      PM_HIP(hipStreamSynchronize(s));
      fprintf(stderr, "[amg bs=%d] level %d transfer + Galerkin product: %.3f s\n", L.bs, l,
              std::chrono::duration<double>(std::chrono::steady_clock::now() - tl0).count());
    }
    if (Ac.n == 0 || Ac.n >= L.n) {
      // coarsening stalled: make this the coarsest level
      Ac.free_all();
      L.P.free_all();
      L.R.free_all();
      dense_inverse(s, L.A, H);
      break;
    }
    cur = Ac;
  }
  H.opcx = nnz_total / nnz0;
  if (prm.cycles > 1) {
    const int64_t m0 = (int64_t)A0.n * A0.bs;
    H.r0 = dalloc<double>(m0);
    H.c0 = dalloc<double>(m0);
    if (prm.fp32) {
      H.r0f = dalloc<float>(m0);
      H.c0f = dalloc<float>(m0);
    }
  }
  if (verbose)
    fprintf(stderr, "[amg bs=%d] %zu levels, coarsest %d unknowns (dense), operator complexity %.3f\n", H.bs,
            H.L.size(), H.ncoarse, H.opcx);
  PM_HIP(hipStreamSynchronize(s));
}

namespace {

template <class T>
__global__ void k_axpy_inplace(int64_t n, const T* __restrict__ a, T* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] += a[i];
}

// x = B b with B = k iterated V-cycles (x_{j+1} = x_j + V (b - A x_j), x_0 = 0);
// the composite is symmetric when V is, so it also serves the transpose.
template <int BS, class T>
void iterated_cycles(hipStream_t s, Hierarchy& H, const T* b, T* x, T* r0, T* c0) {
  using LP = LevelPtrs<BS, T>;
  vcycle_level<BS, T>(s, H, H.prm, 0, b, x);
  Level& L = H.L[0];
  const int64_t m = (int64_t)L.n * BS;
  for (int c = 1; c < H.prm.cycles; ++c) {
    if (BS == 3 && H.lat) {
      lattice_residual<T>(s, H.grid, *H.lat, b, x, r0);
    } else if (BS == 1 && H.cpi) {
      cellpi_residual<T>(s, H.grid, *H.cpi, b, x, r0);
    } else {
      const int nth = L.As.nslices * kSlice;
      k_residual<BS, T><<<blocks_for(nth), kBlock, 0, s>>>(L.n, L.As.sptr, L.As.perm, L.As.col, LP::AV(L.As), b, x,
                                                         r0);
    }
    vcycle_level<BS, T>(s, H, H.prm, 0, r0, c0);
    k_axpy_inplace<T><<<blocks_for(m), kBlock, 0, s>>>(m, c0, x);
    PM_CHECK_LAUNCH();
  }
}

}  // namespace

void amg_vcycle(hipStream_t s, Hierarchy& H, const double* b, double* x) {
  if (H.bs == 3)
    iterated_cycles<3, double>(s, H, b, x, H.r0, H.c0);
  else
    iterated_cycles<1, double>(s, H, b, x, H.r0, H.c0);
}

void amg_vcycle32(hipStream_t s, Hierarchy& H, const float* b, float* x) {
  if (H.bs == 3)
    iterated_cycles<3, float>(s, H, b, x, H.r0f, H.c0f);
  else
    iterated_cycles<1, float>(s, H, b, x, H.r0f, H.c0f);
}

}  // namespace pm
