// Sparse building blocks: device scan, block-CSR <-> sliced-ELL conversion,
// SELL SpMV (FP64 / FP32, block sizes 1 and 3), deterministic transpose,
// row-wise Gustavson SpGEMM with per-wavefront LDS hashing, and inverses of
// the diagonal blocks.  Every result is bitwise reproducible: no
// floating-point atomics; summation orders are fixed.
#include <cstdio>
#include <cstdlib>
#include <iterator>
#include <map>
#include <mutex>
#include <unordered_map>

#include "pm_internal.h"

namespace pm {

// Caching device allocator.  Setup rebuilds many temporaries per step;
// returning freed blocks to per-stream free lists avoids the device-wide
// synchronization of hipFree and repeated hipMalloc calls.  A block freed on
// one stream is only reused by allocations on the same stream, so stream
// order protects kernels still reading it.  A request takes the smallest
// cached block of at least its size class and at most 5/4 of it, so blocks
// of nearby sizes (the data-dependent buffers of the Galerkin products) are
// shared across steps instead of piling up.  When hipMalloc runs out of
// memory, cached blocks are released largest first only until it succeeds.
namespace {
std::mutex g_alloc_mu;
struct Block {
  hipStream_t s;
  size_t bytes;
};
std::unordered_map<hipStream_t, std::multimap<size_t, void*>> g_free;
std::unordered_map<void*, Block> g_live;
size_t g_cached_bytes = 0;
thread_local hipStream_t g_cur_stream = nullptr;

bool alloc_verbose() {
  static const bool v = [] {
    const char* e = getenv("PM_AMG_VERBOSE");
    return e && e[0] == '1';
  }();
  return v;
}

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
    for (auto& e : kv.second) (void)hipFree(e.second);
  g_free.clear();
  g_cached_bytes = 0;
}

// free the largest cached block (of any stream); false if none is left
bool release_largest_locked() {
  std::multimap<size_t, void*>* best = nullptr;
  for (auto& kv : g_free)
    if (!kv.second.empty() && (!best || kv.second.rbegin()->first > best->rbegin()->first)) best = &kv.second;
  if (!best) return false;
  auto last = std::prev(best->end());
  (void)hipFree(last->second);
  g_cached_bytes -= last->first;
  best->erase(last);
  return true;
}
}  // namespace

void set_alloc_stream(hipStream_t s) { g_cur_stream = s; }

void release_device_cache() {
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  release_cached_locked();
}

void* dmalloc(size_t bytes) {
  const size_t cls = size_class(bytes);
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  auto fl = g_free.find(g_cur_stream);
  if (fl != g_free.end()) {
    auto it = fl->second.lower_bound(cls);
    if (it != fl->second.end() && it->first <= cls + cls / 4) {
      void* p = it->second;
      g_cached_bytes -= it->first;
      g_live[p] = Block{g_cur_stream, it->first};
      fl->second.erase(it);
      return p;
    }
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, cls);
  if (e != hipSuccess && alloc_verbose())
    fprintf(stderr, "[alloc] hipMalloc of %zu bytes failed with %zu bytes cached: releasing largest first\n", cls,
            g_cached_bytes);
  while (e != hipSuccess) {
    (void)hipGetLastError();
    if (!release_largest_locked()) break;
    e = hipMalloc(&p, cls);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Error(PM_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
  }
  if (alloc_verbose() && cls >= (size_t(1) << 30))
    fprintf(stderr, "[alloc] new block of %.2f GiB (%.2f GiB cached)\n", cls / 1073741824.0,
            g_cached_bytes / 1073741824.0);
  g_live[p] = Block{g_cur_stream, cls};
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
  g_free[it->second.s].emplace(it->second.bytes, p);
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

void Profiler::end(hipStream_t s, int k, double bytes, double flops) {
  if (!on(k)) return;
  Rec& r = recs[k][used[k]];
  PM_HIP(hipEventRecord(r.b, s));
  r.bytes = bytes;
  r.flops = flops;
  ++used[k];
}

void Profiler::reset(unsigned m) {
  mask = m;
  for (int k = 0; k < kProfCount; ++k) used[k] = 0;
}

void Profiler::collect(int k, int64_t* n, double* ms, double* bytes, double* flops) {
  double t = 0.0, b = 0.0, f = 0.0;
  for (size_t i = 0; i < used[k]; ++i) {
    PM_HIP(hipEventSynchronize(recs[k][i].b));
    float e = 0.0f;
    PM_HIP(hipEventElapsedTime(&e, recs[k][i].a, recs[k][i].b));
    t += e;
    b += recs[k][i].bytes;
    f += recs[k][i].flops;
  }
  *n = (int64_t)used[k];
  *ms = t;
  *bytes = b;
  *flops = f;
}

void Csr::free_all() {
  if (!borrowed) {
    dfree(rowptr);
    dfree(col);
    dfree(val);
    dfree(val32);
  }
  borrowed = false;
  rowptr = nullptr;
  col = nullptr;
  val = nullptr;
  val32 = nullptr;
  n = m = 0;
  nnzb = 0;
}

void Sell::free_all() {
  dfree(sptr);
  dfree(perm);
  dfree(col);
  dfree(val);
  dfree(val32);
  sptr = nullptr;
  perm = nullptr;
  col = nullptr;
  val = nullptr;
  val32 = nullptr;
  n = m = nslices = 0;
  ncols = 0;
  nnzb = 0;
}

namespace {

// ---------------------------------------------------------------------------
// exclusive scan (three phases, 2048 elements per block), int32 or int64
constexpr int kScanT = 256, kScanItems = 8, kScanTile = kScanT * kScanItems;

template <class T>
__global__ void __launch_bounds__(kScanT) k_scan_tiles(const T* __restrict__ in, T* __restrict__ out,
                                                       T* __restrict__ tile_sums, int64_t n) {
  __shared__ T sh[kScanT];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  T v[kScanItems];
  T sum = 0;
  for (int e = 0; e < kScanItems; ++e) {
    const int64_t idx = base + e;
    v[e] = idx < n ? in[idx] : 0;
    sum += v[e];
  }
  sh[threadIdx.x] = sum;
  __syncthreads();
  for (int off = 1; off < kScanT; off <<= 1) {
    const T t = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  T run = sh[threadIdx.x] - sum;  // exclusive prefix of this thread
  for (int e = 0; e < kScanItems; ++e) {
    const int64_t idx = base + e;
    if (idx < n) out[idx] = run;
    run += v[e];
  }
  if (threadIdx.x == kScanT - 1) tile_sums[blockIdx.x] = sh[kScanT - 1];
}

template <class T>
__global__ void __launch_bounds__(1024) k_scan_small(T* __restrict__ a, int n, T* __restrict__ total) {
  // single workgroup exclusive scan of the tile sums (in place)
  __shared__ T sh[1024];
  __shared__ T carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < n; base += 1024) {
    const int idx = base + threadIdx.x;
    const T v = idx < n ? a[idx] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const T t = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
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

template <class T>
__global__ void k_scan_add(T* __restrict__ out, const T* __restrict__ tile_off, int64_t n, const T* __restrict__ total) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < n) out[idx] += tile_off[idx / kScanTile];
  if (idx == 0) out[n] = *total;
}

template <class T>
void scan_impl(hipStream_t s, const T* in, T* out, int64_t n, T* total_host) {
  // out has n+1 entries; out[n] = total
  const int64_t ntiles = (n + kScanTile - 1) / kScanTile;
  T* tiles = dalloc<T>(ntiles + 1);
  T* total = dalloc<T>(1);
  if (n > 0) {
    k_scan_tiles<T><<<(unsigned)ntiles, kScanT, 0, s>>>(in, out, tiles, n);
    PM_CHECK_LAUNCH();
  }
  k_scan_small<T><<<1, 1024, 0, s>>>(tiles, (int)ntiles, total);
  PM_CHECK_LAUNCH();
  k_scan_add<T><<<blocks_for(std::max<int64_t>(n, 1)), kBlock, 0, s>>>(out, tiles, n, total);
  PM_CHECK_LAUNCH();
  // the temporaries go back to this stream's cache: a later allocation on the
  // stream is ordered after these kernels, so only a total read back waits
  if (total_host) {
    PM_HIP(hipMemcpyAsync(total_host, total, sizeof(T), hipMemcpyDeviceToHost, s));
    PM_HIP(hipStreamSynchronize(s));
  }
  dfree(tiles);
  dfree(total);
}

// ---------------------------------------------------------------------------
// CSR -> SELL-C-sigma: within each window of kSellWindow slices the rows are
// sorted by decreasing length (ties by row id), so the rows sharing a slice
// have similar lengths and the padding to the slice width stays small.  The
// kernels find each slot's row in perm; row results are unchanged.
constexpr int kWinRows = kSellWindow * kSlice;  // 512

__global__ void __launch_bounds__(kWinRows) k_sell_perm(const int* __restrict__ rowptr, int n, int* __restrict__ perm) {
  __shared__ uint64_t key[kWinRows];
  const int t = threadIdx.x;
  const int r = blockIdx.x * kWinRows + t;
  // ascending keys = decreasing length, then increasing row; empty slots last
  key[t] = r < n ? ((uint64_t)(0x7FFFFFFF - (rowptr[r + 1] - rowptr[r])) << 32) | (uint32_t)r : ~0ull;
  __syncthreads();
  for (int k = 2; k <= kWinRows; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      const int o = t ^ j;
      if (o > t) {
        const uint64_t a = key[t], b = key[o];
        const bool up = (t & k) == 0;
        if ((a > b) == up) {
          key[t] = b;
          key[o] = a;
        }
      }
      __syncthreads();
    }
  const uint64_t v = key[t];
  perm[blockIdx.x * kWinRows + t] = v == ~0ull ? -1 : (int)(uint32_t)v;
}

__global__ void k_slice_width(const int* __restrict__ rowptr, const int* __restrict__ perm, int n, int nslices,
                              int* __restrict__ w) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nslices) return;
  int mx = 0;
  for (int l = 0; l < kSlice; ++l) {
    const int r = sell_row_of(perm, s * kSlice + l, n);
    if (r >= 0) mx = max(mx, rowptr[r + 1] - rowptr[r]);
  }
  w[s] = mx;
}

template <int BS>
__global__ void k_sell_fill(const int* __restrict__ rowptr, const int* __restrict__ col,
                            const double* __restrict__ val, int n, int m, const int* __restrict__ sptr,
                            const int* __restrict__ perm, int* __restrict__ scol, double* __restrict__ sval,
                            float* __restrict__ sval32) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = t / kSlice, lane = t % kSlice;
  if (s * kSlice >= n) return;
  const int r = sell_row_of(perm, t, n);
  const int c0 = sptr[s], c1 = sptr[s + 1];
  const int b0 = r >= 0 ? rowptr[r] : 0, len = r >= 0 ? rowptr[r + 1] - b0 : 0;
  const int dummy = min(max(r, 0), m - 1);
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
                                                   const int* __restrict__ perm, const int* __restrict__ col,
                                                   const T* __restrict__ val, const T* __restrict__ x,
                                                   T* __restrict__ y) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = t / kSlice, lane = t % kSlice;
  if (s * kSlice >= n) return;
  const int c0 = sptr[s], c1 = sptr[s + 1];
  T acc[BS];
  for (int q = 0; q < BS; ++q) acc[q] = 0;
  sell_row<BS, SellUnroll<BS>::value, T, T>(c0, c1, col, val, x, lane, acc);
  const int r = sell_row_of(perm, t, n);
  if (r >= 0)
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
  scan_impl<int>(s, in, out, n, total_host);
}

void exclusive_scan64(hipStream_t s, const int64_t* in, int64_t* out, int64_t n, int64_t* total_host) {
  scan_impl<int64_t>(s, in, out, n, total_host);
}

void csr_to_sell(hipStream_t s, const Csr& A, Sell& S, bool with_fp32) {
  S.free_all();
  S.bs = A.bs;
  S.n = A.n;
  S.m = A.m;
  S.nslices = (A.n + kSlice - 1) / kSlice;
  S.nnzb = A.nnzb;
  // Sorting pays for 3x3 blocks (rows of 36-72 B per block against a 12-24 B
  // vector entry); for scalar rows the gathers and scatters of the row
  // vectors through perm cost more than the padding saved (measured)
  if (A.bs == 3) {
    const int nwin = (S.nslices + kSellWindow - 1) / kSellWindow;
    S.perm = dalloc<int>((int64_t)nwin * kWinRows);
    if (nwin > 0) k_sell_perm<<<nwin, kWinRows, 0, s>>>(A.rowptr, A.n, S.perm);
  }
  int* w = dalloc<int>(S.nslices);
  k_slice_width<<<blocks_for(S.nslices), kBlock, 0, s>>>(A.rowptr, S.perm, A.n, S.nslices, w);
  PM_CHECK_LAUNCH();
  S.sptr = dalloc<int>(S.nslices + 1);
  int total = 0;
  exclusive_scan(s, w, S.sptr, S.nslices, &total);
  dfree(w);
  S.ncols = total;
  if (const char* v = getenv("PM_AMG_VERBOSE"))
    if (v[0] == '1')
      fprintf(stderr, "[sell] rows %d bs %d: stored %lld of %lld slots (fill %.3f)\n", A.n, A.bs, (long long)A.nnzb,
              (long long)S.ncols * kSlice, (double)S.ncols * kSlice / std::max<int64_t>(1, A.nnzb));
  const int64_t bb = (int64_t)A.bs * A.bs;
  S.col = dalloc<int>(S.ncols * kSlice);
  S.val = dalloc<double>(S.ncols * kSlice * bb);
  S.val32 = with_fp32 ? dalloc<float>(S.ncols * kSlice * bb) : nullptr;
  const int nthreads = S.nslices * kSlice;
  if (A.bs == 3)
    k_sell_fill<3><<<blocks_for(nthreads), kBlock, 0, s>>>(A.rowptr, A.col, A.val, A.n, A.m, S.sptr, S.perm,
                                                           S.col, S.val, S.val32);
  else
    k_sell_fill<1><<<blocks_for(nthreads), kBlock, 0, s>>>(A.rowptr, A.col, A.val, A.n, A.m, S.sptr, S.perm,
                                                           S.col, S.val, S.val32);
  PM_CHECK_LAUNCH();
}

void sell_spmv(hipStream_t s, const Sell& A, const double* x, double* y) {
  const int nthreads = A.nslices * kSlice;
  if (A.bs == 3)
    k_sell_spmv<3, double><<<blocks_for(nthreads), kBlock, 0, s>>>(A.n, A.sptr, A.perm, A.col, A.val, x, y);
  else
    k_sell_spmv<1, double><<<blocks_for(nthreads), kBlock, 0, s>>>(A.n, A.sptr, A.perm, A.col, A.val, x, y);
  PM_CHECK_LAUNCH();
}

void sell_spmv32(hipStream_t s, const Sell& A, const float* x, float* y) {
  const int nthreads = A.nslices * kSlice;
  if (A.bs == 3)
    k_sell_spmv<3, float><<<blocks_for(nthreads), kBlock, 0, s>>>(A.n, A.sptr, A.perm, A.col, A.val32, x, y);
  else
    k_sell_spmv<1, float><<<blocks_for(nthreads), kBlock, 0, s>>>(A.n, A.sptr, A.perm, A.col, A.val32, x, y);
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
  dfree(cnt);
  dfree(tsrc);
  dfree(ttmp);
}

void block_diag_inverse(hipStream_t s, const Csr& A, double* dinv) {
  if (A.bs == 3)
    k_diag_inv<3><<<blocks_for(A.n), kBlock, 0, s>>>(A.n, A.rowptr, A.col, A.val, dinv);
  else
    k_diag_inv<1><<<blocks_for(A.n), kBlock, 0, s>>>(A.n, A.rowptr, A.col, A.val, dinv);
  PM_CHECK_LAUNCH();
}

}  // namespace pm
