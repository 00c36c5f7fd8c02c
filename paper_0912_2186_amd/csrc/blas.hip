// Level-1 vector kernels and deterministic reductions on flat complex
// vectors laid out [nrhs][n] (fine spinors and coarse vectors alike).
//
// Reductions are two-stage and order-fixed: every workgroup reduces its
// grid-stride slice (FP64 accumulation whatever the storage precision) into
// a partial slot; a second small kernel (one workgroup per rhs) sums the
// partials in slot order and writes the result to device memory, so the
// result is bitwise reproducible for a given n and launch shape, and the
// solvers can consume it on the device without a host round trip.  The
// kernel boundary orders the two stages: no device-scope fences or
// same-address atomics, which are expensive across the XCDs' separate L2s.
#include "wmg_internal.h"

namespace wmg {

static constexpr int RB = 256;      // reduction workgroup size
static constexpr int RMAXBLK = 1024; // partial slots per rhs
static constexpr int RSLOT = 32;    // doubles per partial slot

int red_init(Reducer &r, int nrhs_max) {
  r.maxblk = RMAXBLK;
  r.nrhs_max = nrhs_max;
  r.owned = true;
  WMG_HIP(hipMalloc(&r.partial, red_bytes(nrhs_max)));
  return 0;
}

void red_free(Reducer &r) {
  if (r.partial && r.owned) (void)hipFree(r.partial);
  r.partial = nullptr;
}

size_t red_bytes(int nrhs_max) { return sizeof(double) * RSLOT * RMAXBLK * (size_t)nrhs_max; }

void red_attach(Reducer &r, int nrhs_max, double *partial) {
  r.maxblk = RMAXBLK;
  r.nrhs_max = nrhs_max;
  r.partial = partial;
  r.owned = false;
}

// workgroups per rhs of a reduction over np packs (two packs per thread at
// least, at most RMAXBLK)
static int red_blocks(long np) {
  long b = (np + RB * 2 - 1) / (RB * 2);
  if (b < 1) b = 1;
  if (b > RMAXBLK) b = RMAXBLK;
  return (int)b;
}

// sum NC doubles over the workgroup; result valid in thread 0
template <int NC> __device__ __forceinline__ void wg_sum(double v[NC]) {
  __shared__ double sh[NC][RB / 64];
#pragma unroll
  for (int c = 0; c < NC; c++) {
    double x = v[c];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
    v[c] = x;
  }
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int c = 0; c < NC; c++) sh[c][w] = v[c];
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int c = 0; c < NC; c++) {
      double x = 0;
      for (int k = 0; k < RB / 64; k++) x += sh[c][k];
      v[c] = x;
    }
  }
}

// store the workgroup partial (valid in thread 0) into its slot
template <int NC> __device__ __forceinline__ void wg_store(const double v[NC], double *partial, int rhs) {
  if (threadIdx.x == 0) {
    double *p = partial + ((size_t)rhs * RMAXBLK + blockIdx.x) * RSLOT;
#pragma unroll
    for (int c = 0; c < NC; c++) p[c] = v[c];
  }
}

// second stage, one workgroup per rhs: thread t sums slots t, t+RB, ... in
// order for each of the nc values, then a fixed-shape workgroup tree
// combines the threads
__global__ void __launch_bounds__(RB) k_red_final(const double *__restrict__ partial, int nblk, int nc,
                                                 double *__restrict__ out, int out_stride) {
  int rhs = blockIdx.x;
  const double *p = partial + (size_t)rhs * RMAXBLK * RSLOT;
  double v[RSLOT];
#pragma unroll
  for (int c = 0; c < RSLOT; c++) v[c] = 0;
  for (int b = threadIdx.x; b < nblk; b += RB)
#pragma unroll
    for (int c = 0; c < RSLOT; c++)
      if (c < nc) v[c] += p[(size_t)b * RSLOT + c];
  __shared__ double sh[RSLOT][RB / 64];
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < RSLOT; c++) {
    double x = v[c];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
    if (lane == 0 && c < nc) sh[c][w] = x;
  }
  __syncthreads();
  if (threadIdx.x < nc) {
    double x = 0;
    for (int q = 0; q < RB / 64; q++) x += sh[threadIdx.x][q];
    out[(size_t)rhs * out_stride + threadIdx.x] = x;
  }
}

static int red_final(Reducer &R, int nblk, int nc, int nrhs, double *out, int out_stride, hipStream_t st) {
  hipLaunchKernelGGL(k_red_final, dim3(nrhs), dim3(RB), 0, st, (const double *)R.partial, nblk, nc, out, out_stride);
  WMG_HIP(hipGetLastError());
  return 0;
}

__global__ void __launch_bounds__(RB) k_sum_partials(const double *__restrict__ part, long nblk,
                                                    double *__restrict__ out, int out_stride) {
  const int rhs = blockIdx.x;
  const double *p = part + (size_t)rhs * nblk;
  double v[1] = {0};
  for (long b = threadIdx.x; b < nblk; b += RB) v[0] += p[b];
  wg_sum<1>(v);
  if (threadIdx.x == 0) out[(size_t)rhs * out_stride] = v[0];
}

int sum_partials(const double *part, long nblk, int nrhs, double *out, int out_stride, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_partials, dim3(nrhs), dim3(RB), 0, st, part, nblk, out, out_stride);
  WMG_HIP(hipGetLastError());
  return 0;
}

// MODE 0: <x,y> (2), 1: |x|^2 (1), 2: <x,y>,|x|^2 (3)
template <int MODE, class S>
__global__ void __launch_bounds__(RB) k_reduce(const S *__restrict__ x, const S *__restrict__ y, long n,
                                              double *partial) {
  using R = typename store_traits<S>::real;
  constexpr int NC = MODE == 0 ? 2 : (MODE == 1 ? 1 : 3);
  constexpr int PK = pack_len<S>();
  int rhs = blockIdx.y;
  const S *xr = x + (size_t)rhs * n;
  const S *yr = y ? y + (size_t)rhs * n : nullptr;
  double v[NC];
#pragma unroll
  for (int c = 0; c < NC; c++) v[c] = 0;
  const long np = n / PK;
#pragma unroll 4
  for (long i = blockIdx.x * (long)RB + threadIdx.x; i < np; i += (long)gridDim.x * RB) {
    cx<R> a[PK], b[PK];
    ldp<PK>(xr + i * PK, a);
    if (MODE != 1) ldp<PK>(yr + i * PK, b);
#pragma unroll
    for (int e = 0; e < PK; e++) {
      double ar = a[e].re, ai = a[e].im;
      if constexpr (MODE == 1) {
        v[0] += ar * ar + ai * ai;
      } else {
        double br = b[e].re, bi = b[e].im;
        v[0] += ar * br + ai * bi;
        v[1] += ar * bi - ai * br;
        if constexpr (MODE == 2) v[2] += ar * ar + ai * ai;
      }
    }
  }
  wg_sum<NC>(v);
  wg_store<NC>(v, partial, rhs);
}

// per-rhs vector length must hold whole packs
template <class S> static int check_packs(long n, const char *who) {
  if (n % pack_len<S>()) return set_error(-1, "%s: length %ld not a multiple of %d", who, n, pack_len<S>());
  return 0;
}
#define TRY_PK(prec, n, who)                                                     \
  do {                                                                           \
    int e_ = (prec) == P64 ? check_packs<double2>((n), (who)) : check_packs<float2>((n), (who)); \
    if (e_) return e_;                                                           \
  } while (0)

template <int MODE>
static int launch_reduce(Reducer &R, int prec, const void *x, const void *y, long n, int nrhs, double *out,
                         int out_stride, hipStream_t st) {
  if (nrhs > R.nrhs_max) return set_error(-1, "reduction nrhs %d > %d", nrhs, R.nrhs_max);
  TRY_PK(prec, n, "reduction");
  dim3 grid(red_blocks(n / (prec == P64 ? 1 : 2)), nrhs);
  if (prec == P64)
    hipLaunchKernelGGL((k_reduce<MODE, double2>), grid, dim3(RB), 0, st, (const double2 *)x, (const double2 *)y, n,
                       R.partial);
  else
    hipLaunchKernelGGL((k_reduce<MODE, float2>), grid, dim3(RB), 0, st, (const float2 *)x, (const float2 *)y, n,
                       R.partial);
  WMG_HIP(hipGetLastError());
  return red_final(R, (int)grid.x, MODE == 0 ? 2 : (MODE == 1 ? 1 : 3), nrhs, out, out_stride, st);
}

int dot(Reducer &R, int prec, const void *x, const void *y, long n, int nrhs, double *out, int out_stride,
        hipStream_t st) {
  return launch_reduce<0>(R, prec, x, y, n, nrhs, out, out_stride, st);
}
int norm2(Reducer &R, int prec, const void *x, long n, int nrhs, double *out, int out_stride, hipStream_t st) {
  return launch_reduce<1>(R, prec, x, nullptr, n, nrhs, out, out_stride, st);
}
int dot_norm(Reducer &R, int prec, const void *x, const void *y, long n, int nrhs, double *out, int out_stride,
             hipStream_t st) {
  return launch_reduce<2>(R, prec, x, y, n, nrhs, out, out_stride, st);
}

// ---------------------------------------------------------------- multi-dot
// out[rhs][j] = <x_j, y>, j < k (k <= 16), one pass over y
// workgroup sums of nv (<= 32) values into this workgroup's partial slot
template <int NMAX>
__device__ __forceinline__ void wg_store_n(double v[NMAX], int nv, double *partial, int rhs) {
  __shared__ double sh[NMAX][RB / 64];
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < NMAX; c++) {
    double x = v[c];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
    if (lane == 0 && c < nv) sh[c][w] = x;
  }
  __syncthreads();
  if (threadIdx.x < nv) {
    double x = 0;
    for (int q = 0; q < RB / 64; q++) x += sh[threadIdx.x][q];
    partial[((size_t)rhs * RMAXBLK + blockIdx.x) * RSLOT + threadIdx.x] = x;
  }
}

// KT >= k bounds the register arrays (k <= KT, the basis size rounded up
// to 1, 2, 4, 8 or 16)
template <class S, int KT>
__global__ void __launch_bounds__(RB) k_multi_dot(const S *const *__restrict__ xs, int k, const S *__restrict__ y,
                                                 long n, double *partial) {
  using R = typename store_traits<S>::real;
  constexpr int PK = pack_len<S>();
  int rhs = blockIdx.y;
  double v[2 * KT];
#pragma unroll
  for (int c = 0; c < 2 * KT; c++) v[c] = 0;
  const size_t off = (size_t)rhs * n;
  const long np = n / PK;
  for (long i = blockIdx.x * (long)RB + threadIdx.x; i < np; i += (long)gridDim.x * RB) {
    cx<R> b[PK];
    ldp<PK>(y + off + i * PK, b);
#pragma unroll
    for (int j = 0; j < KT; j++) {
      if (j < k) {
        cx<R> a[PK];
        ldp<PK>(xs[j] + off + i * PK, a);
#pragma unroll
        for (int e = 0; e < PK; e++) {
          double ar = a[e].re, ai = a[e].im, br = b[e].re, bi = b[e].im;
          v[2 * j] += ar * br + ai * bi;
          v[2 * j + 1] += ar * bi - ai * br;
        }
      }
    }
  }
  wg_store_n<2 * KT>(v, 2 * k, partial, rhs);
}

static int kt_of(int k) { return k <= 1 ? 1 : (k <= 2 ? 2 : (k <= 4 ? 4 : (k <= 8 ? 8 : 16))); }
#define KT_SWITCH(k, LAUNCH)          \
  switch (kt_of(k)) {                 \
    case 1: { constexpr int KT = 1; LAUNCH; } break;  \
    case 2: { constexpr int KT = 2; LAUNCH; } break;  \
    case 4: { constexpr int KT = 4; LAUNCH; } break;  \
    case 8: { constexpr int KT = 8; LAUNCH; } break;  \
    default: { constexpr int KT = 16; LAUNCH; } break; \
  }

int multi_dot(Reducer &R, int prec, const void *const *xs_dev, int k, const void *y, long n, int nrhs, double *out,
              int out_stride, hipStream_t st) {
  if (k < 1 || k > 16) return set_error(-1, "multi_dot k=%d", k);
  if (nrhs > R.nrhs_max) return set_error(-1, "multi_dot nrhs");
  TRY_PK(prec, n, "multi_dot");
  dim3 grid(red_blocks(n / (prec == P64 ? 1 : 2)), nrhs);
  if (prec == P64)
    KT_SWITCH(k, hipLaunchKernelGGL((k_multi_dot<double2, KT>), grid, dim3(RB), 0, st,
                                    (const double2 *const *)xs_dev, k, (const double2 *)y, n, R.partial))
  else
    KT_SWITCH(k, hipLaunchKernelGGL((k_multi_dot<float2, KT>), grid, dim3(RB), 0, st, (const float2 *const *)xs_dev,
                                    k, (const float2 *)y, n, R.partial))
  WMG_HIP(hipGetLastError());
  return red_final(R, (int)grid.x, 2 * k, nrhs, out, out_stride, st);
}

// ---------------------------------------------------------------- GCR fusions
// Projection step of classical Gram-Schmidt against unnormalised basis
// vectors w_j (|w_j|^2 kept in wn2): b_j = d_j / |w_j|^2, w <- w - sum b_j w_j,
// b_j recorded in beta[j][k] (set_beta: =, else +=).  PASS 1 then reduces
// the new projections <w_j, w> (2k values, the dots of a second pass);
// PASS 2 reduces <w, r> and |w|^2.  One read of every w_j, w (and r).
// gcr_project's pass: 1 and 2 for the two passes of CGS2, 3 for a single
// pass (PASS 2 reductions, beta set).
template <class S, int PASS, int KT>
__global__ void __launch_bounds__(RB) k_gcr_proj(const S *const *__restrict__ W, int k, S *__restrict__ w,
                                                const S *__restrict__ r, const double *__restrict__ d, int dstride,
                                                const double *__restrict__ wn2, int wstride, double *__restrict__ beta,
                                                int bstride, int kcol, long n, double *partial, int set_beta) {
  using R = typename store_traits<S>::real;
  constexpr int PK = pack_len<S>();
  int rhs = blockIdx.y;
  cx<R> b[KT];
#pragma unroll
  for (int j = 0; j < KT; j++) {
    double q = j < k ? wn2[(size_t)rhs * wstride + j] : 0.0;
    double br = (j < k && q > 0) ? d[(size_t)rhs * dstride + 2 * j] / q : 0.0;
    double bi = (j < k && q > 0) ? d[(size_t)rhs * dstride + 2 * j + 1] / q : 0.0;
    b[j] = {(R)br, (R)bi};
    if (blockIdx.x == 0 && threadIdx.x == 0 && j < k) {
      double *bb = beta + (size_t)rhs * bstride + (j * 16 + kcol) * 2;
      if (set_beta) { bb[0] = br; bb[1] = bi; }
      else { bb[0] += br; bb[1] += bi; }
    }
  }
  constexpr int NV = PASS == 1 ? 2 * KT : 3;
  double v[NV];
#pragma unroll
  for (int c = 0; c < NV; c++) v[c] = 0;
  size_t off = (size_t)rhs * n;
  const long np = n / PK;
  for (long i = blockIdx.x * (long)RB + threadIdx.x; i < np; i += (long)gridDim.x * RB) {
    cx<R> wj[KT][PK];
    cx<R> x[PK];
    ldp<PK>(w + off + i * PK, x);
#pragma unroll
    for (int j = 0; j < KT; j++)
      if (j < k) {
        ldp<PK>(W[j] + off + i * PK, wj[j]);
#pragma unroll
        for (int e = 0; e < PK; e++) x[e] = x[e] - b[j] * wj[j][e];
      }
    stp<PK>(w + off + i * PK, x);
    if constexpr (PASS == 1) {
#pragma unroll
      for (int j = 0; j < KT; j++)
        if (j < k)
#pragma unroll
          for (int e = 0; e < PK; e++) {
            v[2 * j] += (double)wj[j][e].re * x[e].re + (double)wj[j][e].im * x[e].im;
            v[2 * j + 1] += (double)wj[j][e].re * x[e].im - (double)wj[j][e].im * x[e].re;
          }
    } else {
      cx<R> rr[PK];
      ldp<PK>(r + off + i * PK, rr);
#pragma unroll
      for (int e = 0; e < PK; e++) {
        v[0] += (double)x[e].re * rr[e].re + (double)x[e].im * rr[e].im;
        v[1] += (double)x[e].re * rr[e].im - (double)x[e].im * rr[e].re;
        v[2] += (double)x[e].re * x[e].re + (double)x[e].im * x[e].im;
      }
    }
  }
  if constexpr (PASS == 2) {
    double t3[3] = {v[0], v[1], v[2]};
    wg_sum<3>(t3);
    wg_store<3>(t3, partial, rhs);
  } else {
    wg_store_n<NV>(v, 2 * k, partial, rhs);
  }
}

int gcr_project(Reducer &R, int prec, int pass, const void *const *W, int k, void *w, const void *r, const double *d,
                int dstride, const double *wn2, int wstride, double *beta, int bstride, int kcol, long n, int nrhs,
                double *out, int out_stride, hipStream_t st) {
  if (k < 1 || k > 16 || nrhs > R.nrhs_max) return set_error(-1, "gcr_project k=%d", k);
  TRY_PK(prec, n, "gcr_project");
  dim3 grid(red_blocks(n / (prec == P64 ? 1 : 2)), nrhs);
#define GP(S, P)                                                                                                  \
  KT_SWITCH(k, hipLaunchKernelGGL((k_gcr_proj<S, P, KT>), grid, dim3(RB), 0, st, (const S *const *)W, k, (S *)w,   \
                                  (const S *)r, d, dstride, wn2, wstride, beta, bstride, kcol, n, R.partial,      \
                                  pass != 2))
  if (prec == P64) { if (pass == 1) { GP(double2, 1); } else { GP(double2, 2); } }
  else { if (pass == 1) { GP(float2, 1); } else { GP(float2, 2); } }
#undef GP
  WMG_HIP(hipGetLastError());
  return red_final(R, (int)grid.x, pass == 1 ? 2 * k : 3, nrhs, out, out_stride, st);
}

// y -= a x (a complex on the device, masked by the caller) and |y|^2
template <class S>
__global__ void __launch_bounds__(RB) k_caxpy_norm(const double *__restrict__ a, int astride, const S *__restrict__ x,
                                                  S *__restrict__ y, long n, double *partial) {
  using R = typename store_traits<S>::real;
  constexpr int PK = pack_len<S>();
  int rhs = blockIdx.y;
  cx<R> c = {(R)(-a[(size_t)rhs * astride]), (R)(-a[(size_t)rhs * astride + 1])};
  size_t off = (size_t)rhs * n;
  double v[1] = {0};
  const long np = n / PK;
#pragma unroll 4
  for (long i = blockIdx.x * (long)RB + threadIdx.x; i < np; i += (long)gridDim.x * RB) {
    cx<R> xv[PK], yv[PK];
    ldp<PK>(x + off + i * PK, xv);
    ldp<PK>(y + off + i * PK, yv);
#pragma unroll
    for (int e = 0; e < PK; e++) {
      yv[e] = cfma(c, xv[e], yv[e]);
      v[0] += (double)yv[e].re * yv[e].re + (double)yv[e].im * yv[e].im;
    }
    stp<PK>(y + off + i * PK, yv);
  }
  wg_sum<1>(v);
  wg_store<1>(v, partial, rhs);
}

int caxpy_norm(Reducer &R, int prec, const double *a, int astride, const void *x, void *y, long n, int nrhs,
               double *out, int out_stride, hipStream_t st) {
  TRY_PK(prec, n, "caxpy_norm");
  dim3 grid(red_blocks(n / (prec == P64 ? 1 : 2)), nrhs);
  if (prec == P64)
    hipLaunchKernelGGL((k_caxpy_norm<double2>), grid, dim3(RB), 0, st, a, astride, (const double2 *)x, (double2 *)y, n,
                       R.partial);
  else
    hipLaunchKernelGGL((k_caxpy_norm<float2>), grid, dim3(RB), 0, st, a, astride, (const float2 *)x, (float2 *)y, n,
                       R.partial);
  WMG_HIP(hipGetLastError());
  return red_final(R, (int)grid.x, 1, nrhs, out, out_stride, st);
}

// ---------------------------------------------------------------- elementwise
// elementwise kernels: one lane per element (pack); a grid-stride loop over
// many elements per lane keeps fewer loads in flight (a plain 1 GiB copy
// streams at 6.2 TB/s one-shot against 4.6-5.5 TB/s grid-stride on MI355X)
static dim3 ew_grid(long n, int nrhs) {
  long b = (n + 255) / 256;
  if (b > (1L << 30) / 256) b = (1L << 30) / 256;
  if (b < 1) b = 1;
  return dim3((unsigned)b, nrhs);
}

template <class A, class B> __host__ __device__ constexpr int pack_len2() {
  return pack_len<A>() > pack_len<B>() ? pack_len<A>() : pack_len<B>();
}

template <class SD, class SS>
__global__ void k_copy(SD *__restrict__ d, const SS *__restrict__ s, long n) {
  using R = typename store_traits<SS>::real;
  constexpr int PK = pack_len2<SD, SS>();
  size_t off = (size_t)blockIdx.y * n;
  const long np = n / PK;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < np; i += (long)gridDim.x * 256) {
    cx<R> v[PK];
    ldp<PK>(s + off + i * PK, v);
    stp<PK>(d + off + i * PK, v);
  }
}

int copy(int pdst, void *dst, int psrc, const void *src, long n, int nrhs, hipStream_t st) {
  if (pdst == P16 || psrc == P16) {
    // FP16 <-> FP32 only, four complex numbers per lane access
    if (n % 4) return set_error(-1, "copy: FP16 length %ld not a multiple of 4", n);
    dim3 g = ew_grid(n / 4, nrhs);
    if (pdst == P32 && psrc == P16)
      hipLaunchKernelGGL((k_copy<float2, __half2>), g, dim3(256), 0, st, (float2 *)dst, (const __half2 *)src, n);
    else if (pdst == P16 && psrc == P32)
      hipLaunchKernelGGL((k_copy<__half2, float2>), g, dim3(256), 0, st, (__half2 *)dst, (const float2 *)src, n);
    else return set_error(-1, "copy: unsupported precision pair %d <- %d", pdst, psrc);
    WMG_HIP(hipGetLastError());
    return 0;
  }
  const int pk = (pdst == P64 && psrc == P64) ? 1 : 2;
  TRY_PK(pk == 1 ? P64 : P32, n, "copy");
  dim3 g = ew_grid(n / pk, nrhs);
  if (pdst == P64 && psrc == P64)
    hipLaunchKernelGGL((k_copy<double2, double2>), g, dim3(256), 0, st, (double2 *)dst, (const double2 *)src, n);
  else if (pdst == P32 && psrc == P64)
    hipLaunchKernelGGL((k_copy<float2, double2>), g, dim3(256), 0, st, (float2 *)dst, (const double2 *)src, n);
  else if (pdst == P64 && psrc == P32)
    hipLaunchKernelGGL((k_copy<double2, float2>), g, dim3(256), 0, st, (double2 *)dst, (const float2 *)src, n);
  else
    hipLaunchKernelGGL((k_copy<float2, float2>), g, dim3(256), 0, st, (float2 *)dst, (const float2 *)src, n);
  WMG_HIP(hipGetLastError());
  return 0;
}

template <class S> __global__ void k_zero(S *__restrict__ x, long n) {
  using R = typename store_traits<S>::real;
  constexpr int PK = pack_len<S>();
  size_t off = (size_t)blockIdx.y * n;
  cx<R> z[PK];
#pragma unroll
  for (int e = 0; e < PK; e++) z[e] = czero<R>();
  const long np = n / PK;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < np; i += (long)gridDim.x * 256) stp<PK>(x + off + i * PK, z);
}

int zero(int prec, void *x, long n, int nrhs, hipStream_t st) {
  if (prec == P16) {
    // n FP16 complex numbers per rhs are n / 2 FP32 complex numbers
    if (n % 4) return set_error(-1, "zero: FP16 length %ld not a multiple of 4", n);
    return zero(P32, x, n / 2, nrhs, st);
  }
  TRY_PK(prec, n, "zero");
  dim3 g = ew_grid(n / (prec == P64 ? 1 : 2), nrhs);
  if (prec == P64) hipLaunchKernelGGL((k_zero<double2>), g, dim3(256), 0, st, (double2 *)x, n);
  else hipLaunchKernelGGL((k_zero<float2>), g, dim3(256), 0, st, (float2 *)x, n);
  WMG_HIP(hipGetLastError());
  return 0;
}

// y += sgn * a * x
template <class S>
__global__ void k_caxpy_dev(const double *__restrict__ a, int astride, double sgn, const S *__restrict__ x,
                            S *__restrict__ y, long n) {
  using R = typename store_traits<S>::real;
  int rhs = blockIdx.y;
  cx<R> c = {(R)(sgn * a[(size_t)rhs * astride]), (R)(sgn * a[(size_t)rhs * astride + 1])};
  size_t off = (size_t)rhs * n;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
    auto xv = ldc(x + off + i);
    auto yv = ldc(y + off + i);
    stc(y + off + i, cfma(c, xv, yv));
  }
}

int caxpy_dev(int prec, const double *a, int astride, double sgn, const void *x, void *y, long n, int nrhs,
              hipStream_t st) {
  dim3 g = ew_grid(n, nrhs);
  if (prec == P64)
    hipLaunchKernelGGL((k_caxpy_dev<double2>), g, dim3(256), 0, st, a, astride, sgn, (const double2 *)x, (double2 *)y, n);
  else
    hipLaunchKernelGGL((k_caxpy_dev<float2>), g, dim3(256), 0, st, a, astride, sgn, (const float2 *)x, (float2 *)y, n);
  WMG_HIP(hipGetLastError());
  return 0;
}

// y = x + sgn * a * y
template <class S>
__global__ void k_cxpay_dev(const S *__restrict__ x, const double *__restrict__ a, int astride, double sgn,
                            S *__restrict__ y, long n) {
  using R = typename store_traits<S>::real;
  int rhs = blockIdx.y;
  cx<R> c = {(R)(sgn * a[(size_t)rhs * astride]), (R)(sgn * a[(size_t)rhs * astride + 1])};
  size_t off = (size_t)rhs * n;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
    auto xv = ldc(x + off + i);
    auto yv = ldc(y + off + i);
    stc(y + off + i, cfma(c, yv, xv));
  }
}

int cxpay_dev(int prec, const void *x, const double *a, int astride, double sgn, void *y, long n, int nrhs,
              hipStream_t st) {
  dim3 g = ew_grid(n, nrhs);
  if (prec == P64)
    hipLaunchKernelGGL((k_cxpay_dev<double2>), g, dim3(256), 0, st, (const double2 *)x, a, astride, sgn, (double2 *)y, n);
  else
    hipLaunchKernelGGL((k_cxpay_dev<float2>), g, dim3(256), 0, st, (const float2 *)x, a, astride, sgn, (float2 *)y, n);
  WMG_HIP(hipGetLastError());
  return 0;
}

// y (+)= sum_j c_j x_j
template <class SY, class SX, int KT>
__global__ void k_multi_caxpy(SY *__restrict__ y, const SX *const *__restrict__ xs, int k, const double *__restrict__ c,
                              int cstride, double sgn, int accumulate, long n) {
  using R = typename store_traits<SY>::real;
  constexpr int PK = pack_len2<SY, SX>();
  int rhs = blockIdx.y;
  size_t off = (size_t)rhs * n;
  cx<R> cc[KT];
#pragma unroll
  for (int j = 0; j < KT; j++)
    cc[j] = j < k ? cx<R>{(R)(sgn * c[(size_t)rhs * cstride + 2 * j]), (R)(sgn * c[(size_t)rhs * cstride + 2 * j + 1])}
                  : czero<R>();
  const long np = n / PK;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < np; i += (long)gridDim.x * 256) {
    cx<R> acc[PK];
    if (accumulate) {
      ldp<PK>(y + off + i * PK, acc);
    } else {
#pragma unroll
      for (int e = 0; e < PK; e++) acc[e] = czero<R>();
    }
#pragma unroll
    for (int j = 0; j < KT; j++)
      if (j < k) {
        cx<R> xv[PK];
        ldp<PK>(xs[j] + off + i * PK, xv);
#pragma unroll
        for (int e = 0; e < PK; e++) acc[e] = cfma(cc[j], xv[e], acc[e]);
      }
    stp<PK>(y + off + i * PK, acc);
  }
}

int multi_caxpy(int py, void *y, int px, const void *const *xs_dev, int k, const double *c, int cstride, double sgn,
                int accumulate, long n, int nrhs, hipStream_t st) {
  if (k < 0 || k > 16) return set_error(-1, "multi_caxpy k=%d", k);
  if (k == 0 && accumulate) return 0;
  if (py == P64 && px == P16) {
    // FP16 x_j (the mixed solve's preconditioner outputs), four per lane
    if (int e_ = check_packs<__half2>(n, "multi_caxpy")) return e_;
    dim3 g = ew_grid(n / 4, nrhs);
    KT_SWITCH(k, hipLaunchKernelGGL((k_multi_caxpy<double2, __half2, KT>), g, dim3(256), 0, st, (double2 *)y,
                                    (const __half2 *const *)xs_dev, k, c, cstride, sgn, accumulate, n))
    WMG_HIP(hipGetLastError());
    return 0;
  }
  const int pk = (py == P64 && px == P64) ? 1 : 2;
  TRY_PK(pk == 1 ? P64 : P32, n, "multi_caxpy");
  dim3 g = ew_grid(n / pk, nrhs);
  if (py == P64 && px == P64)
    KT_SWITCH(k, hipLaunchKernelGGL((k_multi_caxpy<double2, double2, KT>), g, dim3(256), 0, st, (double2 *)y,
                                    (const double2 *const *)xs_dev, k, c, cstride, sgn, accumulate, n))
  else if (py == P64 && px == P32)
    KT_SWITCH(k, hipLaunchKernelGGL((k_multi_caxpy<double2, float2, KT>), g, dim3(256), 0, st, (double2 *)y,
                                    (const float2 *const *)xs_dev, k, c, cstride, sgn, accumulate, n))
  else if (py == P32 && px == P32)
    KT_SWITCH(k, hipLaunchKernelGGL((k_multi_caxpy<float2, float2, KT>), g, dim3(256), 0, st, (float2 *)y,
                                    (const float2 *const *)xs_dev, k, c, cstride, sgn, accumulate, n))
  else
    return set_error(-1, "multi_caxpy precision pair %d %d", py, px);
  WMG_HIP(hipGetLastError());
  return 0;
}

// y = a x + b y (real host scalars)
template <class S> __global__ void k_axpby(double a, const S *__restrict__ x, double b, S *__restrict__ y, long n) {
  using R = typename store_traits<S>::real;
  size_t off = (size_t)blockIdx.y * n;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
    auto xv = ldc(x + off + i), yv = ldc(y + off + i);
    stc(y + off + i, cx<R>{(R)(a * xv.re + b * yv.re), (R)(a * xv.im + b * yv.im)});
  }
}

int axpby(int prec, double a, const void *x, double b, void *y, long n, int nrhs, hipStream_t st) {
  dim3 g = ew_grid(n, nrhs);
  if (prec == P64) hipLaunchKernelGGL((k_axpby<double2>), g, dim3(256), 0, st, a, (const double2 *)x, b, (double2 *)y, n);
  else hipLaunchKernelGGL((k_axpby<float2>), g, dim3(256), 0, st, a, (const float2 *)x, b, (float2 *)y, n);
  WMG_HIP(hipGetLastError());
  return 0;
}

template <class S> __global__ void k_csub(const S *a, const S *b, S *y, long n) {
  size_t off = (size_t)blockIdx.y * n;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256)
    stc(y + off + i, ldc(a + off + i) - ldc(b + off + i));
}

int csub(int prec, const void *a, const void *b, void *y, long n, int nrhs, hipStream_t st) {
  dim3 g = ew_grid(n, nrhs);
  if (prec == P64)
    hipLaunchKernelGGL((k_csub<double2>), g, dim3(256), 0, st, (const double2 *)a, (const double2 *)b, (double2 *)y, n);
  else
    hipLaunchKernelGGL((k_csub<float2>), g, dim3(256), 0, st, (const float2 *)a, (const float2 *)b, (float2 *)y, n);
  WMG_HIP(hipGetLastError());
  return 0;
}

template <class S> __global__ void k_scale_inv_sqrt(S *x, const double *nrm2, int stride, long n, int inv) {
  using R = typename store_traits<S>::real;
  int rhs = blockIdx.y;
  double v = nrm2[(size_t)rhs * stride];
  R f = inv ? (v > 0 ? (R)(1.0 / sqrt(v)) : R(0)) : (R)sqrt(v > 0 ? v : 0.0);
  size_t off = (size_t)rhs * n;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256) stc(x + off + i, f * ldc(x + off + i));
}

static int scale_pow(int prec, void *x, const double *nrm2, int stride, long n, int nrhs, hipStream_t st, int inv) {
  dim3 g = ew_grid(n, nrhs);
  if (prec == P64)
    hipLaunchKernelGGL((k_scale_inv_sqrt<double2>), g, dim3(256), 0, st, (double2 *)x, nrm2, stride, n, inv);
  else hipLaunchKernelGGL((k_scale_inv_sqrt<float2>), g, dim3(256), 0, st, (float2 *)x, nrm2, stride, n, inv);
  WMG_HIP(hipGetLastError());
  return 0;
}
int scale_inv_sqrt(int prec, void *x, const double *nrm2, int stride, long n, int nrhs, hipStream_t st) {
  return scale_pow(prec, x, nrm2, stride, n, nrhs, st, 1);
}
int scale_sqrt(int prec, void *x, const double *nrm2, int stride, long n, int nrhs, hipStream_t st) {
  return scale_pow(prec, x, nrm2, stride, n, nrhs, st, 0);
}

// sigma_3 (coarse) / gamma_5 (fine, AoS view): negate the second half of
// every site's components.  For SoA fine spinors the caller passes nsite=1
// and dof = 12*Vs, which negates components 6..11 of every site.
template <class S> __global__ void k_sigma3(S *x, long nsite, int dof) {
  long n = nsite * dof;
  size_t off = (size_t)blockIdx.y * n;
  int h = dof / 2;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256)
    if ((i % dof) >= h) stc(x + off + i, neg(ldc(x + off + i)));
}

int sigma3(int prec, void *x, long nsite, int dof, int nrhs, hipStream_t st) {
  dim3 g = ew_grid(nsite * dof, nrhs);
  if (prec == P64) hipLaunchKernelGGL((k_sigma3<double2>), g, dim3(256), 0, st, (double2 *)x, nsite, dof);
  else hipLaunchKernelGGL((k_sigma3<float2>), g, dim3(256), 0, st, (float2 *)x, nsite, dof);
  WMG_HIP(hipGetLastError());
  return 0;
}

}  // namespace wmg
