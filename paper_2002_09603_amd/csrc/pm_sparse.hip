// Sparse building blocks: device scan, block-CSR <-> sliced-ELL conversion,
// SELL SpMV (FP64 / FP32, block sizes 1 and 3), deterministic transpose,
// row-wise Gustavson SpGEMM with per-wavefront LDS hashing, and inverses of
// the diagonal blocks.  Every result is bitwise reproducible: no
// floating-point atomics; summation orders are fixed.
#include <mutex>
#include <unordered_map>

#include "pm_internal.h"

namespace pm {

// Caching device allocator.  Setup rebuilds many temporaries per step;
// returning freed blocks to per-(stream, size class) free lists avoids the
// device-wide synchronization of hipFree and repeated hipMalloc calls.  A
// block freed on one stream is only reused by allocations on the same stream,
// so stream order protects kernels still reading it.
namespace {
std::mutex g_alloc_mu;
struct AllocKey {
  hipStream_t s;
  size_t bytes;
  bool operator==(const AllocKey& o) const { return s == o.s && bytes == o.bytes; }
};
struct AllocKeyHash {
  size_t operator()(const AllocKey& k) const { return std::hash<size_t>()(k.bytes) ^ (std::hash<void*>()((void*)k.s) << 1); }
};
std::unordered_map<AllocKey, std::vector<void*>, AllocKeyHash> g_free;
std::unordered_map<void*, AllocKey> g_live;
size_t g_cached_bytes = 0;
thread_local hipStream_t g_cur_stream = nullptr;

size_t size_class(size_t b) {
  if (b <= (1u << 20)) {
    size_t c = 256;
    while (c < b) c <<= 1;
    return c;
  }
  const size_t g = 2u << 20;
  return (b + g - 1) / g * g;
}

void release_cached_locked() {
  for (auto& kv : g_free)
    for (void* p : kv.second) (void)hipFree(p);
  g_free.clear();
  g_cached_bytes = 0;
}
}  // namespace

void set_alloc_stream(hipStream_t s) { g_cur_stream = s; }

void release_device_cache() {
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  release_cached_locked();
}

void* dmalloc(size_t bytes) {
  const AllocKey key{g_cur_stream, size_class(bytes)};
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  auto it = g_free.find(key);
  if (it != g_free.end() && !it->second.empty()) {
    void* p = it->second.back();
    it->second.pop_back();
    g_cached_bytes -= key.bytes;
    g_live[p] = key;
    return p;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, key.bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    release_cached_locked();
    e = hipMalloc(&p, key.bytes);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Error(PM_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
  }
  g_live[p] = key;
  return p;
}

void dfree(void* p) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  auto it = g_live.find(p);
  if (it == g_live.end()) {
    (void)hipFree(p);
    return;
  }
  g_free[it->second].push_back(p);
  g_cached_bytes += it->second.bytes;
  g_live.erase(it);
}

Profiler g_prof;

void Profiler::begin(hipStream_t s, int k) {
  if (!on(k)) return;
  auto& v = recs[k];
  if (used[k] == v.size()) {
    Rec r;
    PM_HIP(hipEventCreate(&r.a));
    PM_HIP(hipEventCreate(&r.b));
    v.push_back(r);
  }
  PM_HIP(hipEventRecord(v[used[k]].a, s));
}

void Profiler::end(hipStream_t s, int k, double bytes) {
  if (!on(k)) return;
  Rec& r = recs[k][used[k]];
  PM_HIP(hipEventRecord(r.b, s));
  r.bytes = bytes;
  ++used[k];
}

void Profiler::reset(unsigned m) {
  mask = m;
  for (int k = 0; k < kProfCount; ++k) used[k] = 0;
}

void Profiler::collect(int k, int64_t* n, double* ms, double* bytes) {
  double t = 0.0, b = 0.0;
  for (size_t i = 0; i < used[k]; ++i) {
    PM_HIP(hipEventSynchronize(recs[k][i].b));
    float e = 0.0f;
    PM_HIP(hipEventElapsedTime(&e, recs[k][i].a, recs[k][i].b));
    t += e;
    b += recs[k][i].bytes;
  }
  *n = (int64_t)used[k];
  *ms = t;
  *bytes = b;
}

void Csr::free_all() {
  dfree(rowptr);
  dfree(col);
  dfree(val);
  rowptr = nullptr;
  col = nullptr;
  val = nullptr;
  n = m = 0;
  nnzb = 0;
}

void Sell::free_all() {
  dfree(sptr);
  dfree(col);
  dfree(val);
  dfree(val32);
  sptr = nullptr;
  col = nullptr;
  val = nullptr;
  val32 = nullptr;
  n = m = nslices = 0;
  ncols = 0;
  nnzb = 0;
}

namespace {

// ---------------------------------------------------------------------------
// exclusive scan of int (three phases, 2048 elements per block)
constexpr int kScanT = 256, kScanItems = 8, kScanTile = kScanT * kScanItems;

__global__ void __launch_bounds__(kScanT) k_scan_tiles(const int* __restrict__ in, int* __restrict__ out,
                                                       int* __restrict__ tile_sums, int n) {
  __shared__ int sh[kScanT];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  int v[kScanItems];
  int sum = 0;
  for (int e = 0; e < kScanItems; ++e) {
    const int64_t idx = base + e;
    v[e] = idx < n ? in[idx] : 0;
    sum += v[e];
  }
  sh[threadIdx.x] = sum;
  __syncthreads();
  for (int off = 1; off < kScanT; off <<= 1) {
    const int t = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  int run = sh[threadIdx.x] - sum;  // exclusive prefix of this thread
  for (int e = 0; e < kScanItems; ++e) {
    const int64_t idx = base + e;
    if (idx < n) out[idx] = run;
    run += v[e];
  }
  if (threadIdx.x == kScanT - 1) tile_sums[blockIdx.x] = sh[kScanT - 1];
}

__global__ void __launch_bounds__(1024) k_scan_small(int* __restrict__ a, int n, int* __restrict__ total) {
  // single workgroup exclusive scan of a (in place), sequential over chunks
  __shared__ int sh[1024];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < n; base += 1024) {
    const int idx = base + threadIdx.x;
    const int v = idx < n ? a[idx] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const int t = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
      __syncthreads();
      sh[threadIdx.x] += t;
      __syncthreads();
    }
    if (idx < n) a[idx] = carry + sh[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry += sh[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ void k_scan_add(int* __restrict__ out, const int* __restrict__ tile_off, int n, int total_pos,
                           const int* __restrict__ total) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < n) out[idx] += tile_off[idx / kScanTile];
  if (idx == 0) out[total_pos] = *total;
}

// ---------------------------------------------------------------------------
// CSR -> SELL
__global__ void k_slice_width(const int* __restrict__ rowptr, int n, int nslices, int* __restrict__ w) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nslices) return;
  int mx = 0;
  for (int l = 0; l < kSlice; ++l) {
    const int r = s * kSlice + l;
    if (r < n) mx = max(mx, rowptr[r + 1] - rowptr[r]);
  }
  w[s] = mx;
}

template <int BS>
__global__ void k_sell_fill(const int* __restrict__ rowptr, const int* __restrict__ col,
                            const double* __restrict__ val, int n, int m, const int* __restrict__ sptr,
                            int* __restrict__ scol, double* __restrict__ sval, float* __restrict__ sval32) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = r / kSlice, lane = r % kSlice;
  if (s * kSlice >= n) return;
  const int c0 = sptr[s], c1 = sptr[s + 1];
  const int b0 = r < n ? rowptr[r] : 0, len = r < n ? rowptr[r + 1] - b0 : 0;
  const int dummy = min(r, m - 1);
  for (int c = c0; c < c1; ++c) {
    const int e = c - c0;
    const size_t slot = (size_t)c * kSlice + lane;
    scol[slot] = e < len ? col[b0 + e] : dummy;
    for (int q = 0; q < BS * BS; ++q) {
      const double v = e < len ? val[(size_t)(b0 + e) * BS * BS + q] : 0.0;
      const size_t vi = ((size_t)c * BS * BS + q) * kSlice + lane;
      sval[vi] = v;
      if (sval32) sval32[vi] = (float)v;
    }
  }
}

// ---------------------------------------------------------------------------
// SELL SpMV: one thread per block row.
template <int BS, class T>
__global__ void __launch_bounds__(256) k_sell_spmv(int n, const int* __restrict__ sptr,
                                                   const int* __restrict__ col, const T* __restrict__ val,
                                                   const T* __restrict__ x, T* __restrict__ y) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = r / kSlice, lane = r % kSlice;
  if (s * kSlice >= n) return;
  const int c0 = sptr[s], c1 = sptr[s + 1];
  T acc[BS];
  for (int q = 0; q < BS; ++q) acc[q] = 0;
  for (int c = c0; c < c1; ++c) {
    const int j = col[(size_t)c * kSlice + lane];
    const T* v = val + (size_t)c * BS * BS * kSlice + lane;
    T xj[BS];
    for (int q = 0; q < BS; ++q) xj[q] = x[(size_t)j * BS + q];
    for (int a = 0; a < BS; ++a)
      for (int b = 0; b < BS; ++b) acc[a] += v[(a * BS + b) * kSlice] * xj[b];
  }
  if (r < n)
    for (int q = 0; q < BS; ++q) y[(size_t)r * BS + q] = acc[q];
}

// plain CSR SpMV (tests, small operators)
template <int BS>
__global__ void k_csr_spmv(int n, const int* __restrict__ rowptr, const int* __restrict__ col,
                           const double* __restrict__ val, const double* __restrict__ x, double* __restrict__ y) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double acc[BS];
  for (int q = 0; q < BS; ++q) acc[q] = 0.0;
  for (int e = rowptr[r]; e < rowptr[r + 1]; ++e) {
    const int j = col[e];
    for (int a = 0; a < BS; ++a)
      for (int b = 0; b < BS; ++b) acc[a] += val[(size_t)e * BS * BS + a * BS + b] * x[(size_t)j * BS + b];
  }
  for (int q = 0; q < BS; ++q) y[(size_t)r * BS + q] = acc[q];
}

// ---------------------------------------------------------------------------
// transpose: count, scan, atomic slot fill, per-row sort by source row
__global__ void k_tr_count(const int* __restrict__ col, int64_t nnz, int* __restrict__ cnt) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nnz) atomicAdd(&cnt[col[e]], 1);
}

__global__ void k_tr_fill(const int* __restrict__ rowptr, const int* __restrict__ col, int n,
                          const int* __restrict__ trow, int* __restrict__ fillc, int* __restrict__ tsrc,
                          int* __restrict__ tcol_tmp) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  for (int e = rowptr[r]; e < rowptr[r + 1]; ++e) {
    const int c = col[e];
    const int p = trow[c] + atomicAdd(&fillc[c], 1);
    tsrc[p] = e;        // source entry
    tcol_tmp[p] = r;    // source row = column in the transpose
  }
}

// one wavefront per transposed row: rank by source row, then move blocks
template <int BS>
__global__ void __launch_bounds__(64) k_tr_sort(const int* __restrict__ trow, const int* __restrict__ tsrc,
                                                const int* __restrict__ tcol_tmp, const double* __restrict__ val,
                                                int* __restrict__ tcol, double* __restrict__ tval, int nt) {
  const int r = blockIdx.x;
  if (r >= nt) return;
  const int p0 = trow[r], p1 = trow[r + 1], len = p1 - p0;
  for (int a = threadIdx.x; a < len; a += 64) {
    const int key = tcol_tmp[p0 + a];
    int rank = 0;
    for (int b = 0; b < len; ++b) rank += tcol_tmp[p0 + b] < key;
    const int src = tsrc[p0 + a];
    tcol[p0 + rank] = key;
    for (int i = 0; i < BS; ++i)
      for (int j = 0; j < BS; ++j)
        tval[(size_t)(p0 + rank) * BS * BS + i * BS + j] = val[(size_t)src * BS * BS + j * BS + i];
  }
}

// ---------------------------------------------------------------------------
// SpGEMM C = A*B (row-wise Gustavson).  Symbolic phase: open-addressing hash
// of the column ids of each product row in LDS.  Two tiers: 4 rows per
// workgroup with 2048-slot tables, then one row per workgroup with 8192-slot
// tables for the rows that overflowed the first tier.
template <int HASH>
__device__ inline int hash_slot(int key) {
  return (int)((unsigned)key * 2654435761u) & (HASH - 1);
}

// Inserts the columns of row `row` of A*B into the wave's table T; keys are
// appended to K (capacity KMAX).  Returns the number of distinct keys, or
// KMAX+1 if the table or the key list overflowed.
template <int HASH, int KMAX>
__device__ int symbolic_row(int row, const int* __restrict__ arp, const int* __restrict__ acol,
                            const int* __restrict__ brp, const int* __restrict__ bcol, int* T, int* K, int* nk,
                            int lane) {
  for (int i = lane; i < HASH; i += 64) T[i] = -1;
  if (lane == 0) *nk = 0;
  __syncthreads();
  for (int e = arp[row]; e < arp[row + 1]; ++e) {
    const int k = acol[e];
    for (int f = brp[k] + lane; f < brp[k + 1]; f += 64) {
      const int key = bcol[f];
      int h = hash_slot<HASH>(key);
      bool placed = false;
      for (int probe = 0; probe < HASH; ++probe) {
        const int prev = atomicCAS(&T[h], -1, key);
        if (prev == -1) {
          const int pos = atomicAdd(nk, 1);
          if (pos < KMAX) K[pos] = key;
          placed = true;
          break;
        }
        if (prev == key) {
          placed = true;
          break;
        }
        h = (h + 1) & (HASH - 1);
      }
      if (!placed) atomicAdd(nk, KMAX + 1);
    }
  }
  __syncthreads();
  const int u = *nk;
  return u > KMAX ? KMAX + 1 : u;
}

template <int KMAX>
__device__ void write_sorted(const int* K, int u, int* __restrict__ dst, int lane) {
  for (int a = lane; a < u; a += 64) {
    const int key = K[a];
    int rank = 0;
    for (int b = 0; b < u; ++b) rank += K[b] < key;
    dst[rank] = key;
  }
}

// tier 1: 4 rows per workgroup.  cnt[row] = distinct columns, or -1 (overflow)
template <bool FILL>
__global__ void __launch_bounds__(256) k_spgemm_sym1(int n, const int* __restrict__ arp, const int* __restrict__ acol,
                                                     const int* __restrict__ brp, const int* __restrict__ bcol,
                                                     int* __restrict__ cnt, const int* __restrict__ crp,
                                                     int* __restrict__ ccol) {
  constexpr int H = 2048, KM = 1536;
  __shared__ int tab[4][H];
  __shared__ int keys[4][KM];
  __shared__ int nk[4];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + w;
  // every wave of the block runs the barriers; rows past n use an empty range
  const bool valid = row < n && (!FILL || cnt[row] >= 0);
  const int r = valid ? row : 0;
  int u;
  if (valid) {
    u = symbolic_row<H, KM>(r, arp, acol, brp, bcol, tab[w], keys[w], &nk[w], lane);
  } else {
    // keep the barrier count uniform across the block
    __syncthreads();
    __syncthreads();
    u = 0;
  }
  if (!valid) return;
  if (!FILL) {
    if (lane == 0) cnt[row] = u > KM ? -1 : u;
  } else {
    write_sorted<KM>(keys[w], u, ccol + crp[row], lane);
  }
}

// tier 2: one row per workgroup, only rows flagged -1 by tier 1
template <bool FILL>
__global__ void __launch_bounds__(64) k_spgemm_sym2(int n, const int* __restrict__ arp, const int* __restrict__ acol,
                                                    const int* __restrict__ brp, const int* __restrict__ bcol,
                                                    const int* __restrict__ flag, int* __restrict__ cnt,
                                                    const int* __restrict__ crp, int* __restrict__ ccol,
                                                    int* __restrict__ status) {
  constexpr int H = 8192, KM = 6144;
  __shared__ int tab[H];
  __shared__ int keys[KM];
  __shared__ int nk;
  const int row = blockIdx.x, lane = threadIdx.x;
  if (row >= n || flag[row] >= 0) return;   // uniform over the block
  const int u = symbolic_row<H, KM>(row, arp, acol, brp, bcol, tab, keys, &nk, lane);
  if (u > KM) {
    if (lane == 0) atomicOr(status, kStatusCapacity);
    return;
  }
  if (!FILL) {
    if (lane == 0) cnt[row] = u;
  } else {
    write_sorted<KM>(keys, u, ccol + crp[row], lane);
  }
}

// Numeric phase: one wavefront per row; A entries in order, lanes over the
// entries of the B row (each output slot is written by one lane per step,
// steps separated by a barrier), so the summation order is fixed.  The row's
// accumulator lives in LDS when it fits, else directly in the output.
template <int BS, int CAP>
__global__ void __launch_bounds__(64) k_spgemm_numeric(int n, const int* __restrict__ arp,
                                                       const int* __restrict__ acol, const double* __restrict__ aval,
                                                       const int* __restrict__ brp, const int* __restrict__ bcol,
                                                       const double* __restrict__ bval, const int* __restrict__ crp,
                                                       const int* __restrict__ ccol, double* __restrict__ cval) {
  __shared__ int cols_l[CAP];
  __shared__ double acc_l[CAP * BS * BS];
  const int row = blockIdx.x, lane = threadIdx.x;
  if (row >= n) return;
  const int c0 = crp[row], u = crp[row + 1] - c0;
  const bool in_lds = u <= CAP;
  const int* cols = in_lds ? (const int*)cols_l : ccol + c0;
  double* acc = in_lds ? (double*)acc_l : cval + (size_t)c0 * BS * BS;
  if (in_lds)
    for (int i = lane; i < u; i += 64) cols_l[i] = ccol[c0 + i];
  for (int i = lane; i < u * BS * BS; i += 64) acc[i] = 0.0;
  __syncthreads();
  for (int e = arp[row]; e < arp[row + 1]; ++e) {
    const int k = acol[e];
    double a[BS * BS];
    for (int q = 0; q < BS * BS; ++q) a[q] = aval[(size_t)e * BS * BS + q];
    for (int f = brp[k] + lane; f < brp[k + 1]; f += 64) {
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
    __syncthreads();
  }
  if (in_lds)
    for (int i = lane; i < u * BS * BS; i += 64) cval[(size_t)c0 * BS * BS + i] = acc[i];
}

// inverse of the diagonal block of every block row
template <int BS>
__global__ void k_diag_inv(int n, const int* __restrict__ rowptr, const int* __restrict__ col,
                           const double* __restrict__ val, double* __restrict__ dinv) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double D[BS * BS];
  for (int q = 0; q < BS * BS; ++q) D[q] = 0.0;
  for (int e = rowptr[r]; e < rowptr[r + 1]; ++e)
    if (col[e] == r)
      for (int q = 0; q < BS * BS; ++q) D[q] = val[(size_t)e * BS * BS + q];
  if (BS == 1) {
    dinv[r] = D[0] != 0.0 ? 1.0 / D[0] : 0.0;
  } else {
    const double c00 = D[4] * D[8] - D[5] * D[7], c01 = D[5] * D[6] - D[3] * D[8], c02 = D[3] * D[7] - D[4] * D[6];
    const double det = D[0] * c00 + D[1] * c01 + D[2] * c02;
    const double id = det != 0.0 ? 1.0 / det : 0.0;
    double* o = dinv + (size_t)r * 9;
    o[0] = c00 * id;
    o[1] = (D[2] * D[7] - D[1] * D[8]) * id;
    o[2] = (D[1] * D[5] - D[2] * D[4]) * id;
    o[3] = c01 * id;
    o[4] = (D[0] * D[8] - D[2] * D[6]) * id;
    o[5] = (D[2] * D[3] - D[0] * D[5]) * id;
    o[6] = c02 * id;
    o[7] = (D[1] * D[6] - D[0] * D[7]) * id;
    o[8] = (D[0] * D[4] - D[1] * D[3]) * id;
  }
}

}  // namespace

void exclusive_scan(hipStream_t s, const int* in, int* out, int n, int* total_host) {
  // out has n+1 entries; out[n] = total
  const int ntiles = (n + kScanTile - 1) / kScanTile;
  int* tiles = dalloc<int>(ntiles + 1);
  int* total = dalloc<int>(1);
  if (n > 0) {
    k_scan_tiles<<<ntiles, kScanT, 0, s>>>(in, out, tiles, n);
    PM_CHECK_LAUNCH();
  }
  k_scan_small<<<1, 1024, 0, s>>>(tiles, ntiles, total);
  PM_CHECK_LAUNCH();
  k_scan_add<<<blocks_for(std::max(n, 1)), kBlock, 0, s>>>(out, tiles, n, n, total);
  PM_CHECK_LAUNCH();
  if (total_host) {
    PM_HIP(hipMemcpyAsync(total_host, total, sizeof(int), hipMemcpyDeviceToHost, s));
    PM_HIP(hipStreamSynchronize(s));
  }
  PM_HIP(hipStreamSynchronize(s));
  dfree(tiles);
  dfree(total);
}

void csr_to_sell(hipStream_t s, const Csr& A, Sell& S, bool with_fp32) {
  S.free_all();
  S.bs = A.bs;
  S.n = A.n;
  S.m = A.m;
  S.nslices = (A.n + kSlice - 1) / kSlice;
  S.nnzb = A.nnzb;
  int* w = dalloc<int>(S.nslices);
  k_slice_width<<<blocks_for(S.nslices), kBlock, 0, s>>>(A.rowptr, A.n, S.nslices, w);
  PM_CHECK_LAUNCH();
  S.sptr = dalloc<int>(S.nslices + 1);
  int total = 0;
  exclusive_scan(s, w, S.sptr, S.nslices, &total);
  dfree(w);
  S.ncols = total;
  const int64_t bb = (int64_t)A.bs * A.bs;
  S.col = dalloc<int>(S.ncols * kSlice);
  S.val = dalloc<double>(S.ncols * kSlice * bb);
  S.val32 = with_fp32 ? dalloc<float>(S.ncols * kSlice * bb) : nullptr;
  const int nthreads = S.nslices * kSlice;
  if (A.bs == 3)
    k_sell_fill<3><<<blocks_for(nthreads), kBlock, 0, s>>>(A.rowptr, A.col, A.val, A.n, A.m, S.sptr, S.col,
                                                           S.val, S.val32);
  else
    k_sell_fill<1><<<blocks_for(nthreads), kBlock, 0, s>>>(A.rowptr, A.col, A.val, A.n, A.m, S.sptr, S.col,
                                                           S.val, S.val32);
  PM_CHECK_LAUNCH();
}

void sell_spmv(hipStream_t s, const Sell& A, const double* x, double* y) {
  const int nthreads = A.nslices * kSlice;
  if (A.bs == 3)
    k_sell_spmv<3, double><<<blocks_for(nthreads), kBlock, 0, s>>>(A.n, A.sptr, A.col, A.val, x, y);
  else
    k_sell_spmv<1, double><<<blocks_for(nthreads), kBlock, 0, s>>>(A.n, A.sptr, A.col, A.val, x, y);
  PM_CHECK_LAUNCH();
}

void sell_spmv32(hipStream_t s, const Sell& A, const float* x, float* y) {
  const int nthreads = A.nslices * kSlice;
  if (A.bs == 3)
    k_sell_spmv<3, float><<<blocks_for(nthreads), kBlock, 0, s>>>(A.n, A.sptr, A.col, A.val32, x, y);
  else
    k_sell_spmv<1, float><<<blocks_for(nthreads), kBlock, 0, s>>>(A.n, A.sptr, A.col, A.val32, x, y);
  PM_CHECK_LAUNCH();
}

void apply_csr(pm_ctx* c, const Csr& A, const double* x, double* y) {
  if (A.bs == 3)
    k_csr_spmv<3><<<blocks_for(A.n), kBlock, 0, c->s>>>(A.n, A.rowptr, A.col, A.val, x, y);
  else
    k_csr_spmv<1><<<blocks_for(A.n), kBlock, 0, c->s>>>(A.n, A.rowptr, A.col, A.val, x, y);
  PM_CHECK_LAUNCH();
}

void csr_transpose(hipStream_t s, const Csr& A, Csr& T) {
  T.free_all();
  T.bs = A.bs;
  T.n = A.m;
  T.m = A.n;
  T.nnzb = A.nnzb;
  int* cnt = dalloc<int>(A.m);
  PM_HIP(hipMemsetAsync(cnt, 0, sizeof(int) * A.m, s));
  if (A.nnzb > 0) {
    k_tr_count<<<blocks_for(A.nnzb), kBlock, 0, s>>>(A.col, A.nnzb, cnt);
    PM_CHECK_LAUNCH();
  }
  T.rowptr = dalloc<int>(A.m + 1);
  exclusive_scan(s, cnt, T.rowptr, A.m, nullptr);
  PM_HIP(hipMemsetAsync(cnt, 0, sizeof(int) * A.m, s));
  int* tsrc = dalloc<int>(A.nnzb);
  int* ttmp = dalloc<int>(A.nnzb);
  k_tr_fill<<<blocks_for(A.n), kBlock, 0, s>>>(A.rowptr, A.col, A.n, T.rowptr, cnt, tsrc, ttmp);
  PM_CHECK_LAUNCH();
  T.col = dalloc<int>(A.nnzb);
  T.val = dalloc<double>(A.nnzb * A.bs * A.bs);
  if (A.m > 0) {
    if (A.bs == 3)
      k_tr_sort<3><<<A.m, 64, 0, s>>>(T.rowptr, tsrc, ttmp, A.val, T.col, T.val, A.m);
    else
      k_tr_sort<1><<<A.m, 64, 0, s>>>(T.rowptr, tsrc, ttmp, A.val, T.col, T.val, A.m);
    PM_CHECK_LAUNCH();
  }
  PM_HIP(hipStreamSynchronize(s));
  dfree(cnt);
  dfree(tsrc);
  dfree(ttmp);
}

void spgemm(hipStream_t s, const Csr& A, const Csr& B, Csr& C) {
  if (A.bs != B.bs || A.m != B.n) throw Error(PM_EINTERNAL, "spgemm: shape mismatch");
  C.free_all();
  C.bs = A.bs;
  C.n = A.n;
  C.m = B.m;
  int* status = dalloc<int>(1);
  PM_HIP(hipMemsetAsync(status, 0, sizeof(int), s));
  int* cnt = dalloc<int>(A.n);
  int* flag = dalloc<int>(A.n);
  const int nb = (A.n + 3) / 4;
  if (A.n > 0) {
    k_spgemm_sym1<false><<<nb, 256, 0, s>>>(A.n, A.rowptr, A.col, B.rowptr, B.col, cnt, nullptr, nullptr);
    PM_CHECK_LAUNCH();
    PM_HIP(hipMemcpyAsync(flag, cnt, sizeof(int) * A.n, hipMemcpyDeviceToDevice, s));
    k_spgemm_sym2<false><<<A.n, 64, 0, s>>>(A.n, A.rowptr, A.col, B.rowptr, B.col, flag, cnt, nullptr, nullptr,
                                            status);
    PM_CHECK_LAUNCH();
  }
  int st = 0;
  PM_HIP(hipMemcpyAsync(&st, status, sizeof(int), hipMemcpyDeviceToHost, s));
  PM_HIP(hipStreamSynchronize(s));
  if (st) {
    dfree(status);
    dfree(cnt);
    dfree(flag);
    throw Error(PM_EINTERNAL, "spgemm: a product row has more distinct columns than the hash capacity");
  }
  C.rowptr = dalloc<int>(A.n + 1);
  int total = 0;
  exclusive_scan(s, cnt, C.rowptr, A.n, &total);
  C.nnzb = total;
  C.col = dalloc<int>(total);
  C.val = dalloc<double>((int64_t)total * A.bs * A.bs);
  if (A.n > 0) {
    k_spgemm_sym1<true><<<nb, 256, 0, s>>>(A.n, A.rowptr, A.col, B.rowptr, B.col, flag, C.rowptr, C.col);
    k_spgemm_sym2<true><<<A.n, 64, 0, s>>>(A.n, A.rowptr, A.col, B.rowptr, B.col, flag, nullptr, C.rowptr, C.col,
                                           status);
    PM_CHECK_LAUNCH();
    if (A.bs == 3)
      k_spgemm_numeric<3, 224><<<A.n, 64, 0, s>>>(A.n, A.rowptr, A.col, A.val, B.rowptr, B.col, B.val, C.rowptr,
                                                  C.col, C.val);
    else
      k_spgemm_numeric<1, 1536><<<A.n, 64, 0, s>>>(A.n, A.rowptr, A.col, A.val, B.rowptr, B.col, B.val,
                                                   C.rowptr, C.col, C.val);
    PM_CHECK_LAUNCH();
  }
  PM_HIP(hipStreamSynchronize(s));
  dfree(cnt);
  dfree(flag);
  dfree(status);
}

void block_diag_inverse(hipStream_t s, const Csr& A, double* dinv) {
  if (A.bs == 3)
    k_diag_inv<3><<<blocks_for(A.n), kBlock, 0, s>>>(A.n, A.rowptr, A.col, A.val, dinv);
  else
    k_diag_inv<1><<<blocks_for(A.n), kBlock, 0, s>>>(A.n, A.rowptr, A.col, A.val, dinv);
  PM_CHECK_LAUNCH();
}

}  // namespace pm
