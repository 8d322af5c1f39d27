// Flexible GMRES (right preconditioning, zero initial guess) in FP64 with
// classical Gram-Schmidt and one re-orthogonalization (CGS2).  Solver
// settings of Sec. 5: stop when ||b - A x||_2 <= rtol ||b||_2.  The
// preconditioner may be the FP32 one (the flexible variant keeps the outer
// recurrence exact in FP64 for a varying inner operator).
//
// Device side: fused multi-dot partial sums (deterministic two-stage
// reductions), multi-AXPY, norms.  Host side: Givens rotations on the small
// Hessenberg column; one device->host copy per iteration.
#include <cmath>

#include "pm_internal.h"

namespace pm {

namespace {

constexpr int kDotBlocks = 2048;  // partial sums per dot product (8 workgroups per CU)
constexpr int kDotGroup = 8;      // basis vectors per multi-dot pass (CGS passes)
constexpr int kDotGroupWide = 24; // basis vectors per multi-dot pass (one-pass Gram-Schmidt)
constexpr int kPartRows = 504;    // rows of the partial-sum buffer (basis vectors + 2 norms)

// part[(i0+g)*kDotBlocks + block] = sum_chunk V_{i0+g} . w for g < cnt <= NG;
// with self_row >= 0 also part[self_row*kDotBlocks + block] = sum_chunk w . w.
// Workgroup sums: shuffles within each wavefront, then the 4 wavefronts in
// order (deterministic).  WAVES waves per SIMD bound the registers so that
// the whole grid is resident at once: NG = 8 with 8 waves and kDotBlocks
// workgroups (the CGS passes); NG = 24 with 4 waves and kDotBlocks / 2
// workgroups reads w once for up to 24 basis vectors (one-pass Gram-Schmidt).
template <int NG, int WAVES>
__global__ void __launch_bounds__(256, WAVES) k_multidot(const double* __restrict__ V, int64_t N, int64_t ld,
                                                         int i0, int cnt, const double* __restrict__ w,
                                                         double* __restrict__ part, int self_row) {
  __shared__ double sh[4][NG + 1];
  double acc[NG + 1];
#pragma unroll
  for (int g = 0; g <= NG; ++g) acc[g] = 0.0;
  const double* Vi = V + (size_t)i0 * ld;
  // element pairs (16-byte loads; vectors start at multiples of ld), then the odd tail
  const int64_t np = N >> 1;
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < np; q += (int64_t)gridDim.x * 256) {
    const int64_t k = 2 * q;
    const double2 wk = *reinterpret_cast<const double2*>(w + k);
#pragma unroll
    for (int g = 0; g < NG; ++g)
      if (g < cnt) {
        const double2 v = *reinterpret_cast<const double2*>(Vi + (size_t)g * ld + k);
        acc[g] += v.x * wk.x + v.y * wk.y;
      }
    acc[NG] += wk.x * wk.x + wk.y * wk.y;
  }
  if ((N & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    const int64_t k = N - 1;
    const double wk = w[k];
    for (int g = 0; g < NG; ++g)
      if (g < cnt) acc[g] += Vi[(size_t)g * ld + k] * wk;
    acc[NG] += wk * wk;
  }
#pragma unroll
  for (int g = 0; g <= NG; ++g)
    for (int off = 32; off > 0; off >>= 1) acc[g] += __shfl_down(acc[g], off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int g = 0; g <= NG; ++g) sh[wave][g] = acc[g];
  __syncthreads();
  if ((int)threadIdx.x <= NG) {
    const int g = threadIdx.x;
    const double v = ((sh[0][g] + sh[1][g]) + sh[2][g]) + sh[3][g];
    if (g < cnt) part[(size_t)(i0 + g) * kDotBlocks + blockIdx.x] = v;
    if (g == NG && self_row >= 0) part[(size_t)self_row * kDotBlocks + blockIdx.x] = v;
  }
}

// h[row0 + i] = sum_{b < np} part[(row0 + i)*kDotBlocks + b], one workgroup per i
__global__ void __launch_bounds__(256) k_dot_final(const double* __restrict__ part, int row0, int cnt, int np,
                                                   double* __restrict__ h) {
  __shared__ double sh[256];
  const int i = blockIdx.x;
  if (i >= cnt) return;
  double s = 0.0;
  for (int b = threadIdx.x; b < np; b += 256) s += part[(size_t)(row0 + i) * kDotBlocks + b];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) h[row0 + i] = sh[0];
}

// w += sign * sum_{i<cnt} coef[i] V_i (coef on the device); with norm_row >= 0
// also part[norm_row*kDotBlocks + block] = sum_chunk w_new . w_new.  V in
// FP64, or FP32 for the preconditioned vectors of the mixed-precision solve.
template <class TV>
struct Vec2;
template <>
struct Vec2<double> {
  using type = double2;
};
template <>
struct Vec2<float> {
  using type = float2;
};

template <class TV>
__global__ void __launch_bounds__(256) k_multiaxpy(const TV* __restrict__ V, int64_t N, int64_t ld, int cnt,
                                                   const double* __restrict__ coef, double* __restrict__ w,
                                                   double sign, double* __restrict__ part, int norm_row) {
  using V2 = typename Vec2<TV>::type;
  __shared__ double c[512];
  __shared__ double sh[256];
  for (int i = threadIdx.x; i < cnt; i += 256) c[i] = coef[i];
  __syncthreads();
  double nn = 0.0;
  const int64_t np = N >> 1;
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < np; q += (int64_t)gridDim.x * 256) {
    const int64_t k = 2 * q;
    double sx = 0.0, sy = 0.0;
    for (int i = 0; i < cnt; ++i) {
      const V2 v = *reinterpret_cast<const V2*>(V + (size_t)i * ld + k);
      sx += c[i] * (double)v.x;
      sy += c[i] * (double)v.y;
    }
    double2 wk = *reinterpret_cast<const double2*>(w + k);
    wk.x += sign * sx;
    wk.y += sign * sy;
    *reinterpret_cast<double2*>(w + k) = wk;
    nn += wk.x * wk.x + wk.y * wk.y;
  }
  if ((N & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    const int64_t k = N - 1;
    double s0 = 0.0;
    for (int i = 0; i < cnt; ++i) s0 += c[i] * (double)V[(size_t)i * ld + k];
    const double wn = w[k] + sign * s0;
    w[k] = wn;
    nn += wn * wn;
  }
  if (norm_row < 0) return;
  sh[threadIdx.x] = nn;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(size_t)norm_row * kDotBlocks + blockIdx.x] = sh[0];
}

__global__ void k_scale_const(int64_t N, const double* __restrict__ w, double s, double* __restrict__ v) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < N) v[k] = w[k] * s;
}

// v = w * s and its FP32 copy vf (the next preconditioner input)
__global__ void k_scale2(int64_t N, const double* __restrict__ w, double s, double* __restrict__ v,
                         float* __restrict__ vf) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const double x = w[k] * s;
  v[k] = x;
  if (vf) vf[k] = (float)x;
}

// scale = 1/sqrt(||w||^2 - ||h||^2) from the projections h[0..nv) and
// h[nv] = ||w||^2 (Pythagoras for the orthogonalised vector); 1 when the
// difference has cancelled below 1e-6 ||w||^2 (the exact norm then rescales)
__global__ void k_pyth_scale(const double* __restrict__ h, int nv, double* __restrict__ scale) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double hh = 0.0;
  for (int i = 0; i < nv; ++i) hh += h[i] * h[i];
  const double b2 = h[nv] - hh;
  scale[0] = (b2 > 1e-6 * h[nv] && b2 > 0.0) ? 1.0 / sqrt(b2) : 1.0;
}

// The same for at most NG basis vectors with the loop over them unrolled so
// that the NG loads of an element pair are issued together: slots past cnt
// reload vector cnt-1 (a cache hit) with coefficient 0, so there is no branch
// and no extra HBM traffic.  Four waves per SIMD, kDotBlocks / 2 workgroups.
template <int NG>
__global__ void __launch_bounds__(256, 4) k_orth_normalize_n(const double* __restrict__ V, int64_t N, int64_t ld,
                                                             int cnt, const double* __restrict__ coef,
                                                             const double* __restrict__ scale,
                                                             const double* __restrict__ w, double* __restrict__ v,
                                                             float* __restrict__ vf, double* __restrict__ part,
                                                             int norm_row) {
  __shared__ double sh[256];
  __shared__ double cl[NG];
  if ((int)threadIdx.x < NG) cl[threadIdx.x] = (int)threadIdx.x < cnt ? coef[threadIdx.x] : 0.0;
  __syncthreads();
  const double sc = scale[0];
  double nn = 0.0;
  const int64_t np = N >> 1;
  const int64_t q0 = (int64_t)blockIdx.x * 256 + threadIdx.x, qs = (int64_t)gridDim.x * 256;
  // per-thread pointers (vector registers), advanced by the grid stride
  const double* pv[NG];
#pragma unroll
  for (int i = 0; i < NG; ++i) pv[i] = V + (size_t)(i < cnt ? i : cnt - 1) * ld + 2 * q0;
  for (int64_t q = q0; q < np; q += qs) {
    const int64_t k = 2 * q;
    double sx = 0.0, sy = 0.0;
#pragma unroll
    for (int i = 0; i < NG; ++i) {
      const double2 x = *reinterpret_cast<const double2*>(pv[i]);
      pv[i] += 2 * qs;
      sx += cl[i] * x.x;
      sy += cl[i] * x.y;
    }
    const double2 wk = *reinterpret_cast<const double2*>(w + k);
    const double wx = wk.x - sx, wy = wk.y - sy;
    nn += wx * wx + wy * wy;
    const double2 out = make_double2(wx * sc, wy * sc);
    *reinterpret_cast<double2*>(v + k) = out;
    if (vf) *reinterpret_cast<float2*>(vf + k) = make_float2((float)out.x, (float)out.y);
  }
  if ((N & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    const int64_t k = N - 1;
    double s0 = 0.0;
    for (int i = 0; i < cnt; ++i) s0 += cl[i] * V[(size_t)i * ld + k];
    const double wn = w[k] - s0;
    nn += wn * wn;
    v[k] = wn * sc;
    if (vf) vf[k] = (float)(wn * sc);
  }
  sh[threadIdx.x] = nn;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(size_t)norm_row * kDotBlocks + blockIdx.x] = sh[0];
}

// v = (w - sum_i coef[i] V_i) * scale[0], optional FP32 copy vf;
// part[norm_row*kDotBlocks + block] = sum_chunk of (w - V coef)^2 (unscaled)
__global__ void __launch_bounds__(256) k_orth_normalize(const double* __restrict__ V, int64_t N, int64_t ld,
                                                        int cnt, const double* __restrict__ coef,
                                                        const double* __restrict__ scale,
                                                        const double* __restrict__ w, double* __restrict__ v,
                                                        float* __restrict__ vf, double* __restrict__ part,
                                                        int norm_row) {
  __shared__ double c[512];
  __shared__ double sh[256];
  for (int i = threadIdx.x; i < cnt; i += 256) c[i] = coef[i];
  __syncthreads();
  const double sc = scale[0];
  double nn = 0.0;
  const int64_t np = N >> 1;
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < np; q += (int64_t)gridDim.x * 256) {
    const int64_t k = 2 * q;
    double sx = 0.0, sy = 0.0;
    for (int i = 0; i < cnt; ++i) {
      const double2 x = *reinterpret_cast<const double2*>(V + (size_t)i * ld + k);
      sx += c[i] * x.x;
      sy += c[i] * x.y;
    }
    const double2 wk = *reinterpret_cast<const double2*>(w + k);
    const double wx = wk.x - sx, wy = wk.y - sy;
    nn += wx * wx + wy * wy;
    const double2 out = make_double2(wx * sc, wy * sc);
    *reinterpret_cast<double2*>(v + k) = out;
    if (vf) *reinterpret_cast<float2*>(vf + k) = make_float2((float)out.x, (float)out.y);
  }
  if ((N & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    const int64_t k = N - 1;
    double s0 = 0.0;
    for (int i = 0; i < cnt; ++i) s0 += c[i] * V[(size_t)i * ld + k];
    const double wn = w[k] - s0;
    nn += wn * wn;
    v[k] = wn * sc;
    if (vf) vf[k] = (float)(wn * sc);
  }
  sh[threadIdx.x] = nn;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(size_t)norm_row * kDotBlocks + blockIdx.x] = sh[0];
}

__global__ void k_sub(int64_t N, const double* __restrict__ b, const double* __restrict__ a, double* __restrict__ r) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < N) r[k] = b[k] - a[k];
}

// sum of squares -> out (two-stage, deterministic)
__global__ void __launch_bounds__(256) k_sq_part(const double* __restrict__ x, int64_t N, double* __restrict__ part) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < N; k += (int64_t)gridDim.x * 256) s += x[k] * x[k];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(256) k_dot_part(const double* __restrict__ x, const double* __restrict__ y,
                                                  int64_t N, double* __restrict__ part) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < N; k += (int64_t)gridDim.x * 256) s += x[k] * y[k];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

int grid_for(int64_t N) { return (int)std::min<int64_t>(kDotBlocks, (N + 255) / 256); }


}  // namespace

// basis V (m+1 FP64 vectors) and the preconditioned vectors: FP64 Z, or FP32
// Zf when they come from the FP32 preconditioner (exactly representable);
// held by the context and grown on demand
static KrylovWs context_ws(pm_ctx* c, int m, bool z32) {
  c->ld = (c->N + 31) / 32 * 32;  // vectors start 256-byte aligned
  if (z32 ? (c->mzf_alloc < m || !c->Zf) : (c->mz_alloc < m || !c->Z)) {
    if (z32) {
      dfree(c->Zf);
      c->Zf = dalloc<float>((int64_t)m * c->ld);
      c->mzf_alloc = m;
    } else {
      dfree(c->Z);
      c->Z = dalloc<double>((int64_t)m * c->ld);
      c->mz_alloc = m;
    }
  }
  if (c->m_alloc < m || !c->V) {
    dfree(c->V);
    c->V = dalloc<double>((int64_t)(m + 1) * c->ld);
    if (!c->red) c->red = dalloc<double>((int64_t)kDotBlocks * kPartRows);
    dfree(c->hcol);
    c->hcol = dalloc<double>(3 * (m + 2) + 8);
    if (c->hhost) (void)hipHostFree(c->hhost);
    c->hhost = nullptr;
    PM_HIP(hipHostMalloc((void**)&c->hhost, sizeof(double) * (m + 8), hipHostMallocDefault));
    c->m_alloc = m;
  }
  KrylovWs w;
  w.m_cap = m;
  w.ld = c->ld;
  w.V = c->V;
  w.Z = z32 ? nullptr : c->Z;
  w.Zf = z32 ? c->Zf : nullptr;
  w.red = c->red;
  w.hcol = c->hcol;
  w.hhost = c->hhost;
  return w;
}

int64_t krylov_ld(int64_t N) { return (N + 31) / 32 * 32; }

// Loads this file's code object onto the current device: one launch of a
// kernel over zero elements (no memory access).  The runtime loads a code
// object at the first launch of one of its kernels and takes device memory
// for it then; pm_setup calls this so that no later solve does.
void krylov_preload(hipStream_t s) {
  k_scale_const<<<1, 64, 0, s>>>(0, nullptr, 1.0, nullptr);
  PM_CHECK_LAUNCH();
}

size_t krylov_device_bytes(int64_t N, int m, bool z32) {
  const auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  const int64_t ld = krylov_ld(N);
  return up(sizeof(double) * (size_t)kDotBlocks * kPartRows) + up(sizeof(double) * (3 * (m + 2) + 8)) +
         up(sizeof(double) * (size_t)(m + 1) * ld) + up((z32 ? sizeof(float) : sizeof(double)) * (size_t)m * ld);
}

KrylovWs krylov_ws_in(void* base, size_t bytes, int64_t N, int m, bool z32) {
  const auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  if (krylov_device_bytes(N, m, z32) > bytes) throw Error(PM_EINVAL, "Krylov workspace does not fit");
  char* p = (char*)base;
  KrylovWs w;
  w.m_cap = m;
  w.ld = krylov_ld(N);
  w.red = (double*)p;
  p += up(sizeof(double) * (size_t)kDotBlocks * kPartRows);
  w.hcol = (double*)p;
  p += up(sizeof(double) * (3 * (m + 2) + 8));
  w.V = (double*)p;
  p += up(sizeof(double) * (size_t)(m + 1) * w.ld);
  if (z32)
    w.Zf = (float*)p;
  else
    w.Z = (double*)p;
  return w;
}

// ||x||^2 into dev[0]; optionally returned to the host (synchronizes)
static double norm_sq(pm_ctx* c, const KrylovWs& w, const double* x, double* dev, bool to_host) {
  const int64_t N = c->N;
  const int gb = grid_for(N);
  k_sq_part<<<gb, 256, 0, c->s>>>(x, N, w.red);
  k_dot_final<<<1, 256, 0, c->s>>>(w.red, 0, 1, gb, dev);
  PM_CHECK_LAUNCH();
  if (!to_host) return 0.0;
  PM_HIP(hipMemcpyAsync(w.hhost, dev, sizeof(double), hipMemcpyDeviceToHost, c->s));
  PM_HIP(hipStreamSynchronize(c->s));
  return w.hhost[0];
}

// One classical Gram-Schmidt pass against V[0..nv): hpass[0..nv) = V^T w,
// w -= V hpass.  With self_norm, hpass[nv] = ||w||^2 before the pass.  The
// partial sums of ||w_new||^2 are left in row nv+1 of the partial buffer.
static void cgs_pass(pm_ctx* c, const KrylovWs& ws, int nv, double* hpass, bool self_norm) {
  const int64_t N = c->N;
  const int gb = grid_for(N);
  for (int i0 = 0; i0 < nv; i0 += kDotGroup) {
    const int cnt = std::min(kDotGroup, nv - i0);
    g_prof.begin(c->s, kProfMultidot);
    k_multidot<kDotGroup, 8><<<gb, 256, 0, c->s>>>(ws.V, N, ws.ld, i0, cnt, c->wvec, ws.red,
                                                   (self_norm && i0 == 0) ? nv : -1);
    g_prof.end(c->s, kProfMultidot, (double)(cnt + 1) * N * 8.0);
  }
  k_dot_final<<<nv + (self_norm ? 1 : 0), 256, 0, c->s>>>(ws.red, 0, nv + (self_norm ? 1 : 0), gb, hpass);
  g_prof.begin(c->s, kProfMultiaxpy);
  k_multiaxpy<double><<<gb, 256, 0, c->s>>>(ws.V, N, ws.ld, nv, hpass, c->wvec, -1.0, ws.red, nv + 1);
  g_prof.end(c->s, kProfMultiaxpy, (double)(nv + 2) * N * 8.0);
  PM_CHECK_LAUNCH();
}

__global__ void k_add_vec(int n, const double* __restrict__ a, double* __restrict__ b) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] += a[i];
}

int fgmres_ws(pm_ctx* c, const KrylovOps& op, const KrylovWs& ws, KrylovHost& hw, const double* b, double* x,
              pm_info* info) {
  const int m = std::max(1, c->opts.restart);
  const int max_it = std::max(1, c->opts.max_it);
  const double rtol = c->opts.rtol;
  if (m > ws.m_cap || m > hw.m_cap) throw Error(PM_EINVAL, "fgmres: restart length exceeds the workspace");
  // one Gram-Schmidt pass: the norm of the new basis vector comes from the
  // projections (Pythagoras) so one pass orthogonalises, normalises and
  // writes the FP32 preconditioner input; the exact norm from the same pass
  // corrects the scale when they differ
  const bool fused = c->opts.orth_passes == 1;
  const bool z32 = fused && op.M32 != nullptr;
  if (z32 ? !ws.Zf : !ws.Z) throw Error(PM_EINTERNAL, "fgmres: workspace lacks the preconditioned vectors");
  const int64_t N = c->N;
  const int64_t ld = ws.ld;
  hipStream_t s = c->s;
  const int gN = blocks_for(N);
  double* h1 = ws.hcol;               // pass-1 coefficients + norm (m+2)
  double* h2 = ws.hcol + (m + 2);     // pass-2 coefficients, then y (m+2)
  double* dev_nrm = ws.hcol + 2 * (m + 2);
  double* dev_scale = dev_nrm + 1;
  double* hhost = ws.hhost;
  float* vf = z32 ? c->pw32 : nullptr;  // FP32 copy of the current basis vector
  double *H = hw.H, *cs = hw.cs, *sn = hw.sn, *g = hw.g, *y = hw.y;
  std::fill(H, H + (size_t)(m + 1) * m, 0.0);
  PM_HIP(hipMemsetAsync(x, 0, sizeof(double) * N, s));
  const double bnorm = std::sqrt(norm_sq(c, ws, b, dev_nrm, true));
  if (!std::isfinite(bnorm)) throw Error(PM_EBREAKDOWN, "fgmres: right-hand side is not finite");
  if (info) {
    info->iters = 0;
    info->relres_est = 0.0;
    info->relres_true = 0.0;
  }
  if (bnorm == 0.0) return PM_OK;
  int its = 0;
  double est = 1.0, relres_true = 1.0, beta = bnorm;
  bool converged = false;
  PM_HIP(hipMemcpyAsync(c->rvec, b, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
  while (true) {
    k_scale2<<<gN, kBlock, 0, s>>>(N, c->rvec, 1.0 / beta, ws.V, vf);
    PM_CHECK_LAUNCH();
    std::fill(g, g + m + 1, 0.0);
    g[0] = beta;
    int jdone = 0;
    for (int j = 0; j < m && its < max_it; ++j) {
      double* vj = ws.V + (size_t)j * ld;
      if (z32) {
        float* zj = ws.Zf + (size_t)j * ld;
        op.M32(vf, zj);
        op.A32(zj, c->wvec);
      } else {
        double* zj = ws.Z + (size_t)j * ld;
        op.M64(vj, zj);
        op.A64(zj, c->wvec);
      }
      const int nv = j + 1;
      double hn;
      if (fused) {
        // h = V^T w and ||w||^2, then v_{j+1} = (w - V h) / ||w - V h|| in one pass
        const int gb = grid_for(N);
        const int gd = std::max(1, std::min(gb, kDotBlocks / 2));
        for (int i0 = 0; i0 < nv; i0 += kDotGroupWide) {
          const int cnt = std::min(kDotGroupWide, nv - i0);
          g_prof.begin(s, kProfMultidot);
          k_multidot<kDotGroupWide, 4><<<gd, 256, 0, s>>>(ws.V, N, ld, i0, cnt, c->wvec, ws.red, i0 == 0 ? nv : -1);
          g_prof.end(s, kProfMultidot, (double)(cnt + 1) * N * 8.0);
        }
        k_dot_final<<<nv + 1, 256, 0, s>>>(ws.red, 0, nv + 1, gd, h1);
        k_pyth_scale<<<1, 64, 0, s>>>(h1, nv, dev_scale);
        g_prof.begin(s, kProfMultiaxpy);
        int go = gb;
        if (nv <= kDotGroupWide) {
          go = gd;
          auto orth = [&](auto ng) {
            constexpr int NG = decltype(ng)::value;
            k_orth_normalize_n<NG><<<go, 256, 0, s>>>(ws.V, N, ld, nv, h1, dev_scale, c->wvec,
                                                      ws.V + (size_t)(j + 1) * ld, vf, ws.red, nv + 1);
          };
          if (nv <= 4)
            orth(std::integral_constant<int, 4>{});
          else if (nv <= 8)
            orth(std::integral_constant<int, 8>{});
          else if (nv <= 16)
            orth(std::integral_constant<int, 16>{});
          else
            orth(std::integral_constant<int, kDotGroupWide>{});
        } else {
          k_orth_normalize<<<go, 256, 0, s>>>(ws.V, N, ld, nv, h1, dev_scale, c->wvec, ws.V + (size_t)(j + 1) * ld,
                                              vf, ws.red, nv + 1);
        }
        g_prof.end(s, kProfMultiaxpy, (double)(nv + 2) * N * 8.0 + (vf ? (double)N * 4.0 : 0.0));
        k_dot_final<<<1, 256, 0, s>>>(ws.red, nv + 1, 1, go, h1);
        PM_CHECK_LAUNCH();
        PM_HIP(hipMemcpyAsync(hhost, h1, sizeof(double) * (nv + 2), hipMemcpyDeviceToHost, s));
        PM_HIP(hipMemcpyAsync(hhost + nv + 2, dev_scale, sizeof(double), hipMemcpyDeviceToHost, s));
        PM_HIP(hipStreamSynchronize(s));
        hn = std::sqrt(hhost[nv + 1]);
        const double sc = hhost[nv + 2];
        if (hn > 0.0 && std::isfinite(hn)) {
          const double prod = hn * sc;  // norm of the written vector
          if (std::fabs(prod - 1.0) > 1e-10) {
            k_scale2<<<gN, kBlock, 0, s>>>(N, ws.V + (size_t)(j + 1) * ld, 1.0 / prod, ws.V + (size_t)(j + 1) * ld,
                                           vf);
            PM_CHECK_LAUNCH();
          } else {
            hn = 1.0 / sc;  // keeps A z_j = V h + hn v_{j+1} exact
          }
        }
      } else {
        // classical Gram-Schmidt, one or two passes; h1[nv+1] = ||w||^2 after them
        cgs_pass(c, ws, nv, h1, false);
        if (c->opts.orth_passes > 1) cgs_pass(c, ws, nv, h2, false);
        k_dot_final<<<1, 256, 0, s>>>(ws.red, nv + 1, 1, grid_for(N), h1);
        if (c->opts.orth_passes > 1) k_add_vec<<<blocks_for(nv), kBlock, 0, s>>>(nv, h2, h1);
        PM_CHECK_LAUNCH();
        PM_HIP(hipMemcpyAsync(hhost, h1, sizeof(double) * (nv + 2), hipMemcpyDeviceToHost, s));
        PM_HIP(hipStreamSynchronize(s));
        hn = std::sqrt(hhost[nv + 1]);
        if (hn > 0.0 && std::isfinite(hn)) {
          k_scale_const<<<gN, kBlock, 0, s>>>(N, c->wvec, 1.0 / hn, ws.V + (size_t)(j + 1) * ld);
          PM_CHECK_LAUNCH();
        }
      }
      bool bad = !std::isfinite(hn);
      for (int i = 0; i < nv; ++i) {
        H[(size_t)i * m + j] = hhost[i];
        bad = bad || !std::isfinite(hhost[i]);
      }
      if (bad) throw Error(PM_EBREAKDOWN, "fgmres: non-finite value in the Arnoldi process");
      H[(size_t)nv * m + j] = hn;
      for (int i = 0; i < j; ++i) {
        const double a = H[(size_t)i * m + j], bb = H[(size_t)(i + 1) * m + j];
        H[(size_t)i * m + j] = cs[i] * a + sn[i] * bb;
        H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * bb;
      }
      const double a = H[(size_t)j * m + j], bb = H[(size_t)(j + 1) * m + j];
      const double den = std::hypot(a, bb);
      cs[j] = den > 0 ? a / den : 1.0;
      sn[j] = den > 0 ? bb / den : 0.0;
      H[(size_t)j * m + j] = den;
      H[(size_t)(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++its;
      jdone = j + 1;
      est = std::fabs(g[j + 1]) / bnorm;
      if (est <= rtol || hn == 0.0) break;
    }
    // y = H^-1 g (upper triangular); x += Z y
    for (int i = jdone - 1; i >= 0; --i) {
      double v = g[i];
      for (int k = i + 1; k < jdone; ++k) v -= H[(size_t)i * m + k] * y[k];
      const double d = H[(size_t)i * m + i];
      if (d == 0.0) throw Error(PM_EBREAKDOWN, "fgmres: singular Hessenberg matrix");
      y[i] = v / d;
    }
    if (jdone > 0) {
      PM_HIP(hipMemcpyAsync(h2, y, sizeof(double) * jdone, hipMemcpyHostToDevice, s));
      if (z32)
        k_multiaxpy<float><<<grid_for(N), 256, 0, s>>>(ws.Zf, N, ld, jdone, h2, x, 1.0, ws.red, -1);
      else
        k_multiaxpy<double><<<grid_for(N), 256, 0, s>>>(ws.Z, N, ld, jdone, h2, x, 1.0, ws.red, -1);
      PM_CHECK_LAUNCH();
    }
    // true residual in FP64; restart from it if needed
    op.A64(x, c->wvec);
    k_sub<<<gN, kBlock, 0, s>>>(N, b, c->wvec, c->rvec);
    PM_CHECK_LAUNCH();
    beta = std::sqrt(norm_sq(c, ws, c->rvec, dev_nrm, true));
    relres_true = beta / bnorm;
    if (!std::isfinite(relres_true)) throw Error(PM_EBREAKDOWN, "fgmres: non-finite residual");
    if (relres_true <= rtol) {
      converged = true;
      break;
    }
    if (its >= max_it || beta == 0.0) break;
  }
  if (info) {
    info->iters = its;
    info->relres_est = est;
    info->relres_true = relres_true;
  }
  return converged ? PM_OK : PM_ENOCONV;
}

KrylovOps step_ops(pm_ctx* c, bool transpose) {
  KrylovOps op;
  op.A64 = [c, transpose](const double* z, double* w) { apply_AH(c, z, w, transpose); };
  op.M64 = [c, transpose](const double* v, double* z) { apply_Minv(c, v, z, transpose); };
  if (c->opts.precond_fp32) {
    op.A32 = [c, transpose](const float* z, double* w) { apply_AH32(c, z, w, transpose); };
    op.M32 = [c, transpose](const float* v, float* z) { apply_Minv32(c, v, z, transpose); };
  }
  return op;
}

int fgmres(pm_ctx* c, const double* b, double* x, bool transpose, pm_info* info) {
  return fgmres_with(c, step_ops(c, transpose), b, x, info);
}

int fgmres_with(pm_ctx* c, const KrylovOps& op, const double* b, double* x, pm_info* info) {
  const int m = std::max(1, c->opts.restart);
  if (m > 500) throw Error(PM_EINVAL, "restart length too large (max 500)");
  const bool z32 = c->opts.orth_passes == 1 && op.M32 != nullptr;
  const KrylovWs ws = context_ws(c, m, z32);
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
  KrylovHost hw{m, H.data(), cs.data(), sn.data(), g.data(), y.data()};
  return fgmres_ws(c, op, ws, hw, b, x, info);
}

}  // namespace pm
