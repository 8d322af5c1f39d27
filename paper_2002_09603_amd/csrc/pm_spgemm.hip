// Sparse matrix-matrix product C = A * B for the Galerkin products of the AMG
// setup (block CSR, square blocks of size 1 or 3), row-wise (Gustavson).
//
// Symbolic: rows are binned by ub = sum over the row of A of the lengths of
// the B rows it touches (an upper bound on the row's distinct columns):
//   small   ub <= 32, <= 64: 32 or 64 lanes per row, one (A entry, B entry)
//                      pair per lane, sorted by a bitonic network
//   medium  ub <= 512  the small configuration first; rows with more than 64
//                      distinct columns are redone with a wavefront per row
//                      and a 1024-slot hash
//   large   otherwise  a wavefront per row, 1024-slot hash first, the rest
//                      with 8192 slots
// Otherwise each group hashes its row's column ids in LDS and ranks the
// distinct ids (sorted order); either way they go to a scratch array at the
// row's ub offset, and a compaction copies them into C after a scan of the
// counts.
// Numeric: rows are binned by their exact number of distinct columns (<= 16:
// 4 lanes per row; <= 64: 16 lanes; <= 512, more: a wavefront per row).  The entries
// of A's row are taken in order; lanes of the group cover the entries of the
// corresponding B row, whose columns are distinct, so each accumulator slot
// has one writer per step and the summation order is fixed (bitwise
// reproducible).  Accumulators live in LDS (large rows fall back to the
// output array when they do not fit).
#include <climits>

#include "pm_internal.h"

namespace pm {

namespace {

enum { kSmallUb = 64, kMediumUb = 512 };

// ub[i] = sum over the entries (i, j) of A of the length of row j of B; G
// lanes per row, summed with shuffles
template <int G>
__global__ void __launch_bounds__(256) k_ub(int n, const int* __restrict__ arp, const int* __restrict__ acol,
                                            const int* __restrict__ brp, int* __restrict__ ub) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = (int)(t / G), l = (int)(t % G);
  int s = 0;
  if (i < n)
    for (int e = arp[i] + l; e < arp[i + 1]; e += G) s += brp[acol[e] + 1] - brp[acol[e]];
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, G);
  if (i < n && l == 0) ub[i] = s;
}

// Row lists per class: class 0 if v <= t0, 1 if v <= t1, 2 if v <= t2,
// else 3.  Counts are aggregated per workgroup (ballots, LDS), one atomic per
// class and workgroup; the order of rows within a list does not affect any
// result.
__global__ void __launch_bounds__(256) k_classify(int n, const int* __restrict__ v, int t0, int t1, int t2,
                                                  int* __restrict__ counters, int* __restrict__ lists) {
  constexpr int NC = 4;
  __shared__ int wcnt[NC][4];
  __shared__ int base[NC];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int c = NC;  // out of range
  if (i < n) {
    const int u = v[i];
    c = u <= t0 ? 0 : (u <= t1 ? 1 : (u <= t2 ? 2 : 3));
  }
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  unsigned long long m[NC];
  for (int k = 0; k < NC; ++k) {
    m[k] = __ballot(c == k);
    if (lane == 0) wcnt[k][wave] = __popcll(m[k]);
  }
  __syncthreads();
  if (threadIdx.x < NC) {
    const int k = threadIdx.x;
    int tot = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += wcnt[k][w];
    base[k] = tot ? atomicAdd(&counters[k], tot) : 0;
  }
  __syncthreads();
  if (c < NC) {
    int off = base[c];
    for (int w = 0; w < wave; ++w) off += wcnt[c][w];
    lists[(size_t)c * n + off + __popcll(m[c] & below)] = i;
  }
}

template <int H>
__device__ inline int hslot(int key) {
  return (int)((unsigned)key * 2654435761u) & (H - 1);
}

// Symbolic phase for one class.  G lanes per row, GPB groups per block,
// hash of H slots, at most KM distinct keys per row.  A row with more keys
// sets cnt[row] = -1 (MARK: to be retried with a larger hash) or the status
// flag.
template <int G, int GPB, int H, int KM, bool MARK = false>
__global__ void __launch_bounds__(G* GPB) k_sym(int nlist, const int* __restrict__ list, const int* __restrict__ arp,
                                                 const int* __restrict__ acol, const int* __restrict__ brp,
                                                 const int* __restrict__ bcol, const int64_t* __restrict__ ubofs,
                                                 int* __restrict__ tmp, int* __restrict__ cnt,
                                                 int* __restrict__ status) {
  constexpr int AMAX = 64;  // entries of A per chunk: their pairs are spread over the lanes
  __shared__ int tab[GPB][H];
  __shared__ int keys[GPB][KM];
  __shared__ int nk[GPB];
  __shared__ int pre_l[GPB][AMAX + 1];
  __shared__ int fb_l[GPB][AMAX];
  const int grp = threadIdx.x / G, lane = threadIdx.x % G;
  const int li = blockIdx.x * GPB + grp;
  // a group (G <= 64 lanes, within one wavefront) shares LDS only with
  // itself: the ordering points below are per wavefront, so groups never
  // synchronize across rows
  if (li >= nlist) return;
  const int row = list[li];
  for (int q = lane; q < H; q += G) tab[grp][q] = -1;
  if (lane == 0) nk[grp] = 0;
  const int e0 = arp[row];
  const int na = arp[row + 1] - e0;
  auto insert = [&](int key) {
    int h = hslot<H>(key);
    for (int probe = 0; probe < H; ++probe) {
      const int prev = atomicCAS(&tab[grp][h], -1, key);
      if (prev == -1) {
        const int pos = atomicAdd(&nk[grp], 1);
        if (pos < KM) keys[grp][pos] = key;
        return;
      }
      if (prev == key) return;
      h = (h + 1) & (H - 1);
    }
    atomicAdd(&nk[grp], KM + 1);
  };
  // the row's entries of A in chunks of AMAX (the set of distinct keys does
  // not depend on the order of insertion)
  for (int cb = 0; cb < na; cb += AMAX) {
    const int nc = min(AMAX, na - cb);
    // B-row extents of the chunk and their prefix sums: each lane takes
    // AMAX/G consecutive entries, sums them, and the lane sums are scanned
    // with shuffles
    {
      constexpr int CH = AMAX / G;
      int len[CH], run = 0;
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int q = lane * CH + u;
        len[u] = 0;
        if (q < nc) {
          const int k = acol[e0 + cb + q];
          const int b0 = brp[k];
          fb_l[grp][q] = b0;
          len[u] = brp[k + 1] - b0;
        }
        run += len[u];
      }
      int incl = run;  // inclusive scan of the lane sums within the group
#pragma unroll
      for (int o = 1; o < G; o <<= 1) {
        const int v = __shfl_up(incl, o, G);
        if (lane >= o) incl += v;
      }
      int acc = incl - run;
      if (lane == 0) pre_l[grp][0] = 0;
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int q = lane * CH + u;
        acc += len[u];
        if (q < nc) pre_l[grp][q + 1] = acc;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
    // the (entry of A, entry of its B row) pairs of the chunk, spread over the lanes
    const int* pre = pre_l[grp];
    const int tot = pre[nc];
    for (int pq = lane; pq < tot; pq += G) {
      int lo = 0, hi = nc - 1;  // largest e with pre[e] <= pq
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= pq) lo = mid; else hi = mid - 1;
      }
      insert(bcol[fb_l[grp][lo] + (pq - pre[lo])]);
    }
    // every lane's reads of the staging arrays precede the next chunk's writes
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
  const int u = nk[grp];
  if (u > KM) {
    if (lane == 0) {
      if (MARK)
        cnt[row] = -1;
      else
        atomicOr(status, kStatusCapacity);
    }
    return;
  }
  int* dst = tmp + ubofs[row];
  for (int a = lane; a < u; a += G) {
    const int key = keys[grp][a];
    int rank = 0;
    for (int b = 0; b < u; ++b) rank += keys[grp][b] < key;
    dst[rank] = key;
  }
  if (lane == 0) cnt[row] = u;
}

// Symbolic phase for rows with at most G (A entry, B entry) pairs, G lanes
// per row and one pair per lane: lane q takes pair q (the pairs of A's entries
// in order, located by a scan of the B-row lengths and a search over the
// lanes), the G column ids are sorted by a bitonic network over the lanes and
// the distinct ones written in ascending order (the output of k_sym, without
// LDS or atomics).
template <int G>
__global__ void __launch_bounds__(256) k_sym_sort(int nlist, const int* __restrict__ list,
                                                  const int* __restrict__ arp, const int* __restrict__ acol,
                                                  const int* __restrict__ brp, const int* __restrict__ bcol,
                                                  const int64_t* __restrict__ ubofs, int* __restrict__ tmp,
                                                  int* __restrict__ cnt) {
  static_assert(G == 32 || G == 64, "one row per half or whole wavefront");
  constexpr int LG = G == 32 ? 5 : 6;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int li = (int)(t / G), l = (int)(t % G);
  const bool valid = li < nlist;
  const int row = valid ? list[li] : 0;
  const int e0 = valid ? arp[row] : 0, na = valid ? arp[row + 1] - e0 : 0;
  int key = INT_MAX;
  int base = 0;  // pairs of the earlier chunks of A entries
  for (int c0 = 0; c0 < na; c0 += G) {  // the same trip count on every lane of the row
    const int q = c0 + l;
    int fb = 0, len = 0;
    if (q < na) {
      const int k = acol[e0 + q];
      fb = brp[k];
      len = brp[k + 1] - fb;
    }
    int incl = len;
#pragma unroll
    for (int o = 1; o < G; o <<= 1) {
      const int v = __shfl_up(incl, o, G);
      if (l >= o) incl += v;
    }
    const int total = __shfl(incl, G - 1, G);
    const int p = l - base;  // this lane's pair within the chunk, if 0 <= p < total
    int lo = 0, hi = G - 1;  // first entry lane whose inclusive count exceeds p
#pragma unroll
    for (int it = 0; it < LG; ++it) {
      const int mid = (lo + hi) >> 1;
      const int v = __shfl(incl, mid, G);
      if (v > p) hi = mid; else lo = mid + 1;
      if (lo > hi) lo = hi;
    }
    const int fbj = __shfl(fb, lo, G), exj = __shfl(incl - len, lo, G);
    if (p >= 0 && p < total) key = bcol[fbj + p - exj];
    base += total;
  }
  // bitonic sort (ascending) over the G lanes of the row
#pragma unroll
  for (int k = 2; k <= G; k <<= 1)
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const int other = __shfl_xor(key, j, G);
      const bool up = (l & k) == 0;
      const bool lower = (l & j) == 0;
      key = (lower == up) ? min(key, other) : max(key, other);
    }
  const int prev = __shfl_up(key, 1, G);
  const bool first = key != INT_MAX && (l == 0 || prev != key);
  const int lane = threadIdx.x & 63, gbase = lane & ~(G - 1);
  const unsigned long long gmask = (G == 64) ? ~0ull : ((1ull << G) - 1ull);
  const unsigned long long grp = (__ballot(first) >> gbase) & gmask;
  if (valid) {
    if (first) tmp[ubofs[row] + __popcll(grp & ((1ull << l) - 1ull))] = key;
    if (l == 0) cnt[row] = __popcll(grp);
  }
}

// rows of a list whose symbolic pass overflowed (cnt = -1)
__global__ void k_retry_list(int nlist, const int* __restrict__ list, const int* __restrict__ cnt,
                             int* __restrict__ counter, int* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nlist) return;
  const int row = list[i];
  if (cnt[row] < 0) out[atomicAdd(counter, 1)] = row;
}

// copy the sorted keys of each row from the scratch (ub offsets) into C
__global__ void k_compact(int n, const int64_t* __restrict__ ubofs, const int* __restrict__ tmp,
                          const int* __restrict__ crp, int* __restrict__ ccol) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int row = (int)(t >> 4), lane = (int)(t & 15);
  if (row >= n) return;
  const int c0 = crp[row], u = crp[row + 1] - c0;
  const int* src = tmp + ubofs[row];
  for (int a = lane; a < u; a += 16) ccol[c0 + a] = src[a];
}

// Numeric phase for one class: G lanes per row, GPB groups per block, LDS
// accumulator of CAP blocks per group.  Rows wider than CAP (large class
// only) accumulate in the output array instead.
template <int BS, int G, int GPB, int CAP>
__global__ void __launch_bounds__(G* GPB) k_num(int nlist, const int* __restrict__ list, const int* __restrict__ arp,
                                                 const int* __restrict__ acol, const double* __restrict__ aval,
                                                 const int* __restrict__ brp, const int* __restrict__ bcol,
                                                 const double* __restrict__ bval, const int* __restrict__ crp,
                                                 const int* __restrict__ ccol, double* __restrict__ cval) {
  __shared__ int cols_l[GPB][CAP];
  __shared__ double acc_l[GPB][CAP * BS * BS];
  const int grp = threadIdx.x / G, lane = threadIdx.x % G;
  const int li = blockIdx.x * GPB + grp;
  if (li >= nlist) return;  // groups never synchronize across rows: per-wave ordering only
  const int row = list[li];
  const int c0 = crp[row], u = crp[row + 1] - c0;
  const bool in_lds = u <= CAP;
  const int* cols = in_lds ? (const int*)cols_l[grp] : ccol + c0;
  double* acc = in_lds ? (double*)acc_l[grp] : cval + (size_t)c0 * BS * BS;
  if (in_lds)
    for (int i = lane; i < u; i += G) cols_l[grp][i] = ccol[c0 + i];
  for (int i = lane; i < u * BS * BS; i += G) acc[i] = 0.0;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
  for (int e = arp[row]; e < arp[row + 1]; ++e) {
    const int k = acol[e];
    double a[BS * BS];
    for (int q = 0; q < BS * BS; ++q) a[q] = aval[(size_t)e * BS * BS + q];
    for (int f = brp[k] + lane; f < brp[k + 1]; f += G) {
      const int key = bcol[f];
      int lo = 0, hi = u - 1;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (cols[mid] < key) lo = mid + 1; else hi = mid;
      }
      double* dst = acc + (size_t)lo * BS * BS;
      const double* b = bval + (size_t)f * BS * BS;
      for (int i = 0; i < BS; ++i)
        for (int j = 0; j < BS; ++j) {
          double sacc = dst[i * BS + j];
          for (int t = 0; t < BS; ++t) sacc += a[i * BS + t] * b[t * BS + j];
          dst[i * BS + j] = sacc;
        }
    }
    // the next entry of A may update the same slots from other lanes
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
  }
  if (in_lds)
    for (int i = lane; i < u * BS * BS; i += G) cval[(size_t)c0 * BS * BS + i] = acc[i];
}

// Numeric phase for rows with at most CAP <= 64 distinct columns, G lanes
// per row, 64/G rows per wavefront (the LDS accumulators are sized by CAP:
// the rows of the Galerkin products of the block operator mostly have <= 16,
// and the smaller footprint keeps more wavefronts resident).  Same order of
// summation as k_num (entries of A in order, lanes over the B row), with the
// latency of the dependent loads hidden: the B-row extents of the next AMAX
// entries of the A row are staged in LDS, and the B-row entries and A block of
// the next entry are loaded while the current one is accumulated.  G = 4 suits
// A P_smoothed (prolongator rows of ~4 blocks), G = 16 the restriction
// R (A P) (rows of A P of ~16 blocks).
template <int BS>
__device__ inline int slot_in(const int* __restrict__ cols, int u, int key) {
  int lo = 0, hi = u - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (cols[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

template <int BS, int CAP, int G>
__global__ void __launch_bounds__(64) k_num_small(int nlist, const int* __restrict__ list,
                                                  const int* __restrict__ arp, const int* __restrict__ acol,
                                                  const double* __restrict__ aval, const int* __restrict__ brp,
                                                  const int* __restrict__ bcol, const double* __restrict__ bval,
                                                  const int* __restrict__ crp, const int* __restrict__ ccol,
                                                  double* __restrict__ cval) {
  constexpr int GPB = 64 / G, AMAX = 32, B2 = BS * BS;
  __shared__ int cols_l[GPB][CAP];
  __shared__ double acc_l[GPB][CAP * B2];
  __shared__ int fb_l[GPB][AMAX];
  __shared__ int fe_l[GPB][AMAX];
  const int grp = threadIdx.x / G, lane = threadIdx.x % G;
  const int li = blockIdx.x * GPB + grp;
  if (li >= nlist) return;  // groups never synchronize across rows: per-wave ordering only
  const int row = list[li];
  const int c0 = crp[row], u = crp[row + 1] - c0;
  const int e0 = arp[row], na = arp[row + 1] - e0;
  for (int i = lane; i < u; i += G) cols_l[grp][i] = ccol[c0 + i];
  for (int i = lane; i < u * B2; i += G) acc_l[grp][i] = 0.0;
  // Two register sets alternate (loop unrolled by two): the operands of entry
  // e+1 are loaded, with clamped always-valid indices, before entry e is
  // accumulated, and no register copies tie the loads to the loop back edge.
  struct Ops {
    int fb, fe, key;
    bool v;
    double a[B2], b[B2];
  };
  // entries cb .. cb+nc-1 of the row, their extents staged
  int cb = 0, nc = 0;
  auto load = [&](int e, Ops& o) {
    const int ec = min(e, nc - 1);
    o.fb = fb_l[grp][ec];
    o.fe = fe_l[grp][ec];
    o.v = (e < nc) && (o.fb + lane < o.fe);
    const int fs = o.v ? o.fb + lane : 0;
    o.key = bcol[fs];
    for (int q = 0; q < B2; ++q) {
      o.a[q] = aval[(size_t)(e0 + cb + ec) * B2 + q];
      o.b[q] = bval[(size_t)fs * B2 + q];
    }
  };
  auto accumulate = [&](const Ops& o) {
    if (o.v) {
      double* dst = &acc_l[grp][slot_in<BS>(cols_l[grp], u, o.key) * B2];
      for (int i = 0; i < BS; ++i)
        for (int j = 0; j < BS; ++j) {
          double sacc = dst[i * BS + j];
          for (int t = 0; t < BS; ++t) sacc += o.a[i * BS + t] * o.b[t * BS + j];
          dst[i * BS + j] = sacc;
        }
    }
    // B rows longer than the group (rare): remaining entries, in order
    for (int f = o.fb + lane + G; f < o.fe; f += G) {
      double* dst = &acc_l[grp][slot_in<BS>(cols_l[grp], u, bcol[f]) * B2];
      const double* bb = bval + (size_t)f * B2;
      for (int i = 0; i < BS; ++i)
        for (int j = 0; j < BS; ++j) {
          double sacc = dst[i * BS + j];
          for (int t = 0; t < BS; ++t) sacc += o.a[i * BS + t] * bb[t * BS + j];
          dst[i * BS + j] = sacc;
        }
    }
    // the next entry of A may update the same slots from other lanes of this
    // wavefront: LDS accesses of one wavefront complete in order, so only the
    // compiler must not move them across this point
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  };
  for (cb = 0; cb < na; cb += AMAX) {
    nc = min(AMAX, na - cb);
    // B-row extents of this chunk of the row's A entries (the previous
    // chunk's reads of the staging arrays precede this in wavefront order)
    for (int q = lane; q < nc; q += G) {
      const int k = acol[e0 + cb + q];
      fb_l[grp][q] = brp[k];
      fe_l[grp][q] = brp[k + 1];
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
    Ops p0, p1;
    load(0, p0);
    for (int e = 0; e < nc; e += 2) {
      load(e + 1, p1);
      accumulate(p0);
      if (e + 1 >= nc) break;
      load(e + 2, p0);
      accumulate(p1);
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
  for (int i = lane; i < u * B2; i += G) cval[(size_t)c0 * B2 + i] = acc_l[grp][i];
}

// classes by the exact number of distinct columns: <= 16, <= 64, <= 512, more
template <int BS>
void numeric_launch(hipStream_t s, const int* counts, const int* lists, int n, const Csr& A, const Csr& B, Csr& C) {
  if (counts[0] > 0)
    k_num_small<BS, 16, 4><<<(counts[0] + 15) / 16, 64, 0, s>>>(counts[0], lists, A.rowptr, A.col, A.val, B.rowptr,
                                                               B.col, B.val, C.rowptr, C.col, C.val);
  if (counts[1] > 0)
    k_num_small<BS, 64, 16><<<(counts[1] + 3) / 4, 64, 0, s>>>(counts[1], lists + (size_t)n, A.rowptr, A.col,
                                                               A.val, B.rowptr, B.col, B.val, C.rowptr, C.col,
                                                               C.val);
  if (counts[2] > 0)
    k_num<BS, 64, 1, 512><<<counts[2], 64, 0, s>>>(counts[2], lists + 2 * (size_t)n, A.rowptr, A.col, A.val,
                                                   B.rowptr, B.col, B.val, C.rowptr, C.col, C.val);
  if (counts[3] > 0)
    k_num<BS, 64, 1, (BS == 3 ? 224 : 1536)><<<counts[3], 64, 0, s>>>(counts[3], lists + 3 * (size_t)n, A.rowptr,
                                                                       A.col, A.val, B.rowptr, B.col, B.val,
                                                                       C.rowptr, C.col, C.val);
  PM_CHECK_LAUNCH();
}

// Numeric phase when B is a tentative prolongator (row j: one identity block
// in column agg[j], none if agg[j] < 0): C[i, K] = sum of A[i, j] over the
// entries with agg[j] == K, in entry order.  G lanes per row, each owning
// every G-th output column of the row.
template <int BS, int G>
__global__ void __launch_bounds__(256) k_num_ptent(int n, const int* __restrict__ arp, const int* __restrict__ acol,
                                                   const double* __restrict__ aval, const int* __restrict__ agg,
                                                   const int* __restrict__ crp, const int* __restrict__ ccol,
                                                   double* __restrict__ cval) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int row = (int)(t / G), lane = (int)(t % G);
  if (row >= n) return;
  const int c0 = crp[row], u = crp[row + 1] - c0;
  const int e0 = arp[row], e1 = arp[row + 1];
  for (int q = lane; q < u; q += G) {
    const int key = ccol[c0 + q];
    double acc[BS * BS];
    for (int k = 0; k < BS * BS; ++k) acc[k] = 0.0;
    for (int e = e0; e < e1; ++e)
      if (agg[acol[e]] == key)
        for (int k = 0; k < BS * BS; ++k) acc[k] += aval[(size_t)e * BS * BS + k];
    for (int k = 0; k < BS * BS; ++k) cval[(size_t)(c0 + q) * BS * BS + k] = acc[k];
  }
}

// Products with the tentative prolongator (one entry per aggregated row,
// column = aggregate): the pattern of row i of A P_tent is the sorted set of
// distinct agg[j] >= 0 over the entries (i, j) of A.  G lanes per row, rows of
// at most G entries: a bitonic sort of the row's keys across the lanes, then
// the first of each run is kept.  The keys go to tmp at A's row offsets.
// longest row: per-workgroup maxima (grid-stride, 256 threads), then one workgroup
__global__ void __launch_bounds__(256) k_row_len_part(int n, const int* __restrict__ rp, int* __restrict__ part) {
  __shared__ int sh[4];
  int v = 0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) v = max(v, rp[i + 1] - rp[i]);
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = max(max(sh[0], sh[1]), max(sh[2], sh[3]));
}

__global__ void __launch_bounds__(256) k_max_final(int np, const int* __restrict__ part, int* __restrict__ out) {
  __shared__ int sh[4];
  int v = 0;
  for (int i = threadIdx.x; i < np; i += 256) v = max(v, part[i]);
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) *out = max(max(sh[0], sh[1]), max(sh[2], sh[3]));
}

template <int G>
__global__ void __launch_bounds__(256) k_sym_ptent(int n, const int* __restrict__ arp, const int* __restrict__ acol,
                                                   const int* __restrict__ agg, int* __restrict__ tmp,
                                                   int* __restrict__ cnt) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int row = (int)(t / G), l = (int)(t % G);
  int key = INT_MAX;
  int e0 = 0;
  if (row < n) {
    e0 = arp[row];
    if (l < arp[row + 1] - e0) {
      const int a = agg[acol[e0 + l]];
      if (a >= 0) key = a;
    }
  }
  // bitonic sort (ascending) over the G lanes of the row
#pragma unroll
  for (int k = 2; k <= G; k <<= 1)
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const int other = __shfl_xor(key, j, G);
      const bool up = (l & k) == 0;
      const bool lower = (l & j) == 0;
      key = (lower == up) ? min(key, other) : max(key, other);
    }
  const int prev = __shfl_up(key, 1, G);
  const bool first = key != INT_MAX && (l == 0 || prev != key);
  const int lane = threadIdx.x & 63, base = lane & ~(G - 1);
  const unsigned long long gmask = (G == 64) ? ~0ull : ((1ull << G) - 1ull);
  const unsigned long long grp = (__ballot(first) >> base) & gmask;
  if (row < n) {
    if (first) tmp[e0 + __popcll(grp & ((1ull << l) - 1ull))] = key;
    if (l == 0) cnt[row] = __popcll(grp);
  }
}

// copy the sorted keys of each row from the scratch (int offsets) into C
__global__ void k_compact32(int n, const int* __restrict__ ofs, const int* __restrict__ tmp,
                            const int* __restrict__ crp, int* __restrict__ ccol) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int row = (int)(t >> 4), lane = (int)(t & 15);
  if (row >= n) return;
  const int c0 = crp[row], u = crp[row + 1] - c0;
  const int* src = tmp + ofs[row];
  for (int a = lane; a < u; a += 16) ccol[c0 + a] = src[a];
}

__global__ void k_i64_from_i32(int n, const int* __restrict__ a, int64_t* __restrict__ b) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

}  // namespace

void spgemm(hipStream_t s, const Csr& A, const Csr& B, Csr& C, const int* ptent_agg) {
  if (A.bs != B.bs || A.m != B.n) throw Error(PM_EINTERNAL, "spgemm: shape mismatch");
  C.free_all();
  C.bs = A.bs;
  C.n = A.n;
  C.m = B.m;
  const int n = A.n;
  C.rowptr = dalloc<int>(n + 1);
  if (n == 0) {
    PM_HIP(hipMemsetAsync(C.rowptr, 0, sizeof(int), s));
    C.nnzb = 0;
    C.col = dalloc<int>(0);
    C.val = dalloc<double>(0);
    return;
  }
  if (ptent_agg) {
    // rows of at most 64 entries: the sort-based pattern of A P_tent
    const int np = (int)std::min<int64_t>(1024, blocks_for(n));
    int* mx = dalloc<int>(np + 1);
    k_row_len_part<<<np, 256, 0, s>>>(n, A.rowptr, mx + 1);
    k_max_final<<<1, 256, 0, s>>>(np, mx + 1, mx);
    PM_CHECK_LAUNCH();
    int maxna = 0;
    PM_HIP(hipMemcpyAsync(&maxna, mx, sizeof(int), hipMemcpyDeviceToHost, s));
    PM_HIP(hipStreamSynchronize(s));
    dfree(mx);
    if (maxna <= 64) {
      int* tmp = dalloc<int>(std::max<int64_t>(A.nnzb, 1));
      int* cnt = dalloc<int>(n);
      auto sym = [&](auto g) {
        constexpr int G = decltype(g)::value;
        k_sym_ptent<G><<<blocks_for((int64_t)n * G), kBlock, 0, s>>>(n, A.rowptr, A.col, ptent_agg, tmp, cnt);
      };
      if (maxna <= 16)
        sym(std::integral_constant<int, 16>{});
      else if (maxna <= 32)
        sym(std::integral_constant<int, 32>{});
      else
        sym(std::integral_constant<int, 64>{});
      PM_CHECK_LAUNCH();
      int total = 0;
      exclusive_scan(s, cnt, C.rowptr, n, &total);
      C.nnzb = total;
      C.col = dalloc<int>(total);
      C.val = dalloc<double>((int64_t)total * A.bs * A.bs);
      k_compact32<<<blocks_for((int64_t)n * 16), kBlock, 0, s>>>(n, A.rowptr, tmp, C.rowptr, C.col);
      if (A.bs == 3)
        k_num_ptent<3, 8><<<blocks_for((int64_t)n * 8), kBlock, 0, s>>>(n, A.rowptr, A.col, A.val, ptent_agg,
                                                                        C.rowptr, C.col, C.val);
      else
        k_num_ptent<1, 8><<<blocks_for((int64_t)n * 8), kBlock, 0, s>>>(n, A.rowptr, A.col, A.val, ptent_agg,
                                                                        C.rowptr, C.col, C.val);
      PM_CHECK_LAUNCH();
      dfree(tmp);
      dfree(cnt);
      return;
    }
  }
  int* ub = dalloc<int>(n);
  int* counters = dalloc<int>(5);
  int* lists = dalloc<int>(4 * (int64_t)n);
  int64_t* ub64 = dalloc<int64_t>(n);
  int64_t* ubofs = dalloc<int64_t>(n + 1);
  int* cnt = dalloc<int>(n);
  PM_HIP(hipMemsetAsync(counters, 0, 5 * sizeof(int), s));
  if ((double)A.nnzb <= 12.0 * n)
    k_ub<4><<<blocks_for((int64_t)n * 4), kBlock, 0, s>>>(n, A.rowptr, A.col, B.rowptr, ub);
  else
    k_ub<16><<<blocks_for((int64_t)n * 16), kBlock, 0, s>>>(n, A.rowptr, A.col, B.rowptr, ub);
  k_classify<<<blocks_for(n), kBlock, 0, s>>>(n, ub, kSmallUb / 2, kSmallUb, kMediumUb, counters, lists);
  k_i64_from_i32<<<blocks_for(n), kBlock, 0, s>>>(n, ub, ub64);
  PM_CHECK_LAUNCH();
  int h[4] = {0, 0, 0, 0};
  int64_t tmp_total = 0;
  PM_HIP(hipMemcpyAsync(h, counters, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
  exclusive_scan64(s, ub64, ubofs, n, &tmp_total);
  int* tmp = dalloc<int>(std::max<int64_t>(tmp_total, 1));
  int* status = counters + 4;  // cleared above
  // bounds <= 32 and <= 64: one pair per lane, sorted
  if (h[0] > 0)
    k_sym_sort<32><<<blocks_for((int64_t)h[0] * 32), kBlock, 0, s>>>(h[0], lists, A.rowptr, A.col, B.rowptr, B.col,
                                                                    ubofs, tmp, cnt);
  if (h[1] > 0)
    k_sym_sort<64><<<blocks_for((int64_t)h[1] * 64), kBlock, 0, s>>>(h[1], lists + (size_t)n, A.rowptr, A.col,
                                                                    B.rowptr, B.col, ubofs, tmp, cnt);
  // Rows with a larger bound mostly have few distinct columns (Galerkin rows):
  // each class first tries the next smaller configuration, marking the rows
  // that do not fit (cnt = -1), which are redone with its own.
  int* rc = dalloc<int>(2);
  int* retry = dalloc<int>(std::max(h[2], h[3]));
  PM_HIP(hipMemsetAsync(rc, 0, 2 * sizeof(int), s));
  auto retry_rows = [&](const int* rl, int nl, int* counter) {
    k_retry_list<<<blocks_for(nl), kBlock, 0, s>>>(nl, rl, cnt, counter, retry);
    PM_CHECK_LAUNCH();
    int nr = 0;
    PM_HIP(hipMemcpyAsync(&nr, counter, sizeof(int), hipMemcpyDeviceToHost, s));
    PM_HIP(hipStreamSynchronize(s));
    return nr;
  };
  if (h[2] > 0) {
    const int* rl = lists + 2 * (size_t)n;
    k_sym<16, 16, 128, 64, true><<<(h[2] + 15) / 16, 256, 0, s>>>(h[2], rl, A.rowptr, A.col, B.rowptr, B.col,
                                                                  ubofs, tmp, cnt, status);
    const int nr = retry_rows(rl, h[2], rc);
    if (nr > 0)
      k_sym<64, 4, 1024, 512><<<(nr + 3) / 4, 256, 0, s>>>(nr, retry, A.rowptr, A.col, B.rowptr, B.col, ubofs, tmp,
                                                           cnt, status);
    PM_CHECK_LAUNCH();
  }
  if (h[3] > 0) {
    // the 1024-slot hash first, the rest with 8192
    const int* rl = lists + 3 * (size_t)n;
    k_sym<64, 4, 1024, 512, true><<<(h[3] + 3) / 4, 256, 0, s>>>(h[3], rl, A.rowptr, A.col, B.rowptr, B.col, ubofs,
                                                                 tmp, cnt, status);
    const int nr = retry_rows(rl, h[3], rc + 1);
    if (nr > 0)
      k_sym<64, 1, 8192, 6144><<<nr, 64, 0, s>>>(nr, retry, A.rowptr, A.col, B.rowptr, B.col, ubofs, tmp, cnt,
                                                 status);
    PM_CHECK_LAUNCH();
  }
  dfree(rc);
  dfree(retry);
  PM_CHECK_LAUNCH();
  int st = 0;
  PM_HIP(hipMemcpyAsync(&st, status, sizeof(int), hipMemcpyDeviceToHost, s));
  PM_HIP(hipStreamSynchronize(s));
  if (st) {
    for (void* p : {(void*)ub, (void*)counters, (void*)lists, (void*)ub64, (void*)ubofs, (void*)cnt, (void*)tmp})
      dfree(p);
    throw Error(PM_EINTERNAL, "spgemm: a product row has more distinct columns than the hash capacity");
  }
  int total = 0;
  exclusive_scan(s, cnt, C.rowptr, n, &total);
  C.nnzb = total;
  C.col = dalloc<int>(total);
  C.val = dalloc<double>((int64_t)total * A.bs * A.bs);
  k_compact<<<blocks_for((int64_t)n * 16), kBlock, 0, s>>>(n, ubofs, tmp, C.rowptr, C.col);
  if (ptent_agg) {
    if (A.bs == 3)
      k_num_ptent<3, 8><<<blocks_for((int64_t)n * 8), kBlock, 0, s>>>(n, A.rowptr, A.col, A.val, ptent_agg,
                                                                      C.rowptr, C.col, C.val);
    else
      k_num_ptent<1, 8><<<blocks_for((int64_t)n * 8), kBlock, 0, s>>>(n, A.rowptr, A.col, A.val, ptent_agg,
                                                                      C.rowptr, C.col, C.val);
    PM_CHECK_LAUNCH();
    for (void* p : {(void*)ub, (void*)counters, (void*)lists, (void*)ub64, (void*)ubofs, (void*)cnt, (void*)tmp})
      dfree(p);
    return;
  }
  // numeric phase binned by the exact number of distinct columns
  PM_HIP(hipMemsetAsync(counters, 0, 4 * sizeof(int), s));
  k_classify<<<blocks_for(n), kBlock, 0, s>>>(n, cnt, 16, 64, 512, counters, lists);
  PM_CHECK_LAUNCH();
  PM_HIP(hipMemcpyAsync(h, counters, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
  PM_HIP(hipStreamSynchronize(s));
  if (A.bs == 3)
    numeric_launch<3>(s, h, lists, n, A, B, C);
  else
    numeric_launch<1>(s, h, lists, n, A, B, C);
  for (void* p : {(void*)ub, (void*)counters, (void*)lists, (void*)ub64, (void*)ubofs, (void*)cnt, (void*)tmp})
    dfree(p);
}

}  // namespace pm
