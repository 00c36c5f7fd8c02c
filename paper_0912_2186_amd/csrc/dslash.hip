// Wilson-Dirac operator (arXiv:0912.2186, Sec. 2, Eq. 2.2):
//   out(x) = (4+m) in(x) - 1/2 sum_mu [ (1-gamma_mu) U_mu(x)     in(x+mu)
//                                     + (1+gamma_mu) U_mu(x-mu)^dag in(x-mu) ]
// in the chiral basis gamma_mu = [[0, A_mu], [A_mu^dag, 0]] (A_1..3 = -i sigma_k,
// A_4 = 1), where (1 -+ gamma_mu) psi = [h; -+A_mu^dag h] with
// h = psi_up -+ A_mu psi_down: each hop multiplies only a two-spin half
// spinor by the 3x3 link and rebuilds the lower spins from it.
//
// One thread per site (and per tile of RT right-hand sides, which then share
// every link load).  Links and spinors are stored component-major with sites
// fastest, so each load instruction of a wavefront reads consecutive
// addresses; neighbour reuse is left to L2/MALL, with workgroups mapped so
// that each XCD sweeps one contiguous range of sites.
#include "wmg_internal.h"

namespace wmg {

// h = psi_up - S * A_mu psi_down   (S = +1: 1-gamma, S = -1: 1+gamma)
template <int MU, int S, class R> __device__ __forceinline__ void project(const cx<R> p[12], cx<R> h[6]) {
#pragma unroll
  for (int c = 0; c < 3; c++) {
    cx<R> p0 = p[c], p1 = p[3 + c], p2 = p[6 + c], p3 = p[9 + c];
    cx<R> a0, a1;  // A_mu psi_down
    if (MU == 0) { a0 = times_mi(p3); a1 = times_mi(p2); }
    if (MU == 1) { a0 = neg(p3); a1 = p2; }
    if (MU == 2) { a0 = times_mi(p2); a1 = times_i(p3); }
    if (MU == 3) { a0 = p2; a1 = p3; }
    if (S > 0) { h[c] = p0 - a0; h[3 + c] = p1 - a1; }
    else { h[c] = p0 + a0; h[3 + c] = p1 + a1; }
  }
}

// acc_up += g; acc_down += -S * A_mu^dag g
template <int MU, int S, class R> __device__ __forceinline__ void reconstruct(const cx<R> g[6], cx<R> acc[12]) {
#pragma unroll
  for (int c = 0; c < 3; c++) {
    cx<R> g0 = g[c], g1 = g[3 + c];
    acc[c] = acc[c] + g0;
    acc[3 + c] = acc[3 + c] + g1;
    cx<R> b0, b1;  // A_mu^dag g
    if (MU == 0) { b0 = times_i(g1); b1 = times_i(g0); }
    if (MU == 1) { b0 = g1; b1 = neg(g0); }
    if (MU == 2) { b0 = times_i(g0); b1 = times_mi(g1); }
    if (MU == 3) { b0 = g0; b1 = g1; }
    if (S > 0) { acc[6 + c] = acc[6 + c] - b0; acc[9 + c] = acc[9 + c] - b1; }
    else { acc[6 + c] = acc[6 + c] + b0; acc[9 + c] = acc[9 + c] + b1; }
  }
}

// g = U h (DAG = 0) or U^dag h (DAG = 1) on both half-spinor spins
template <int DAG, class R> __device__ __forceinline__ void su3_mul(const cx<R> u[9], const cx<R> h[6], cx<R> g[6]) {
#pragma unroll
  for (int sp = 0; sp < 2; sp++)
#pragma unroll
    for (int a = 0; a < 3; a++) {
      cx<R> acc = czero<R>();
#pragma unroll
      for (int b = 0; b < 3; b++) {
        if (DAG == 0) acc = cfma(u[3 * a + b], h[3 * sp + b], acc);
        else acc = cfmac(u[3 * b + a], h[3 * sp + b], acc);
      }
      g[3 * sp + a] = acc;
    }
}

// ---------------------------------------------------------------- SoA
template <class TL, class TS, int RT>
__global__ void __launch_bounds__(256) k_wilson_soa(const TL *__restrict__ U, const TS *__restrict__ in,
                                                   TS *__restrict__ out, int L0, int L1, int L2, int L3, long V,
                                                   float diagf, double diagd, int nrhs) {
  using R = typename store_traits<TS>::real;
  const R diag = sizeof(R) == 8 ? (R)diagd : (R)diagf;
  // tiles = (site tile, rhs tile) with the rhs tile fastest, so the rhs
  // tiles of one site tile run back to back on one XCD and share its links
  int nrt = (nrhs + RT - 1) / RT;
  long ntile = (V + 255) / 256 * nrt;
  long tile = xcd_tile(blockIdx.x, gridDim.x);
  if (tile >= ntile) return;
  long s = (tile / nrt) * 256 + threadIdx.x;
  if (s >= V) return;
  int r0 = (int)(tile % nrt) * RT;
  const int L[4] = {L0, L1, L2, L3};
  int x[4];
  site_coords(L, s, x);
  long stride[4] = {1, (long)L0, (long)L0 * L1, (long)L0 * L1 * L2};
  cx<R> acc[RT][12];
#pragma unroll
  for (int t = 0; t < RT; t++)
#pragma unroll
    for (int c = 0; c < 12; c++) acc[t][c] = czero<R>();

  auto load_link = [&](int mu, long site, cx<R> u[9]) {
#pragma unroll
    for (int e = 0; e < 9; e++) {
      auto v = ldc(U + ((size_t)(mu * 9 + e)) * V + site);
      u[e] = {(R)v.re, (R)v.im};
    }
  };
  auto load_psi = [&](int r, long site, cx<R> p[12]) {
#pragma unroll
    for (int c = 0; c < 12; c++) {
      auto v = ldc(in + ((size_t)r * 12 + c) * V + site);
      p[c] = {(R)v.re, (R)v.im};
    }
  };

#define WILSON_DIR(MU)                                                                         \
  {                                                                                            \
    long fw = x[MU] == L[MU] - 1 ? s - (long)(L[MU] - 1) * stride[MU] : s + stride[MU];        \
    long bw = x[MU] == 0 ? s + (long)(L[MU] - 1) * stride[MU] : s - stride[MU];                \
    cx<R> u[9], p[12], h[6], g[6];                                                             \
    load_link(MU, s, u);                                                                       \
    _Pragma("unroll") for (int t = 0; t < RT; t++) {                                           \
      if (r0 + t < nrhs) {                                                                     \
        load_psi(r0 + t, fw, p);                                                               \
        project<MU, 1>(p, h);                                                                  \
        su3_mul<0>(u, h, g);                                                                   \
        reconstruct<MU, 1>(g, acc[t]);                                                         \
      }                                                                                        \
    }                                                                                          \
    load_link(MU, bw, u);                                                                      \
    _Pragma("unroll") for (int t = 0; t < RT; t++) {                                           \
      if (r0 + t < nrhs) {                                                                     \
        load_psi(r0 + t, bw, p);                                                               \
        project<MU, -1>(p, h);                                                                 \
        su3_mul<1>(u, h, g);                                                                   \
        reconstruct<MU, -1>(g, acc[t]);                                                        \
      }                                                                                        \
    }                                                                                          \
  }
  WILSON_DIR(0)
  WILSON_DIR(1)
  WILSON_DIR(2)
  WILSON_DIR(3)
#undef WILSON_DIR

#pragma unroll
  for (int t = 0; t < RT; t++) {
    if (r0 + t >= nrhs) continue;
    cx<R> p[12];
    load_psi(r0 + t, s, p);
#pragma unroll
    for (int c = 0; c < 12; c++) {
      cx<R> o = {diag * p[c].re - R(0.5) * acc[t][c].re, diag * p[c].im - R(0.5) * acc[t][c].im};
      stc(out + ((size_t)(r0 + t) * 12 + c) * V + s, o);
    }
  }
}

template <class TL, class TS>
static void launch_soa(const Geom &g, const void *U, double m, const void *in, void *out, int nrhs, hipStream_t st) {
  constexpr int RT = sizeof(TS) == 16 ? 1 : 2;
  long ntile = (g.V + 255) / 256 * ((nrhs + RT - 1) / RT);
  dim3 grid((unsigned)xcd_grid(ntile));
  hipLaunchKernelGGL((k_wilson_soa<TL, TS, RT>), grid, dim3(256), 0, st, (const TL *)U, (const TS *)in, (TS *)out,
                     g.L[0], g.L[1], g.L[2], g.L[3], g.V, (float)(4.0 + m), 4.0 + m, nrhs);
}

int wilson_soa(const Geom &g, int lprec, const void *U, int sprec, double m, const void *in, void *out, int nrhs,
               hipStream_t st) {
  if (sprec == P64 && lprec == P64) launch_soa<double2, double2>(g, U, m, in, out, nrhs, st);
  else if (sprec == P32 && lprec == P32) launch_soa<float2, float2>(g, U, m, in, out, nrhs, st);
  else if (sprec == P32 && lprec == P16) launch_soa<__half2, float2>(g, U, m, in, out, nrhs, st);
  else return set_error(-1, "wilson_soa: unsupported precision pair link=%d spinor=%d", lprec, sprec);
  WMG_HIP(hipGetLastError());
  return 0;
}

// ---------------------------------------------------------------- canonical
// FP64, canonical AoS layouts of the C ABI: U[s][mu][a][b], psi[s][12].
__global__ void __launch_bounds__(256) k_wilson_canon(const double2 *__restrict__ U, const double2 *__restrict__ in,
                                                     double2 *__restrict__ out, int L0, int L1, int L2, int L3, long V,
                                                     double diag) {
  long s = blockIdx.x * 256L + threadIdx.x;
  if (s >= V) return;
  const int L[4] = {L0, L1, L2, L3};
  int x[4];
  site_coords(L, s, x);
  long stride[4] = {1, (long)L0, (long)L0 * L1, (long)L0 * L1 * L2};
  cx<double> acc[12];
#pragma unroll
  for (int c = 0; c < 12; c++) acc[c] = czero<double>();
#define CANON_DIR(MU)                                                                   \
  {                                                                                     \
    long fw = x[MU] == L[MU] - 1 ? s - (long)(L[MU] - 1) * stride[MU] : s + stride[MU]; \
    long bw = x[MU] == 0 ? s + (long)(L[MU] - 1) * stride[MU] : s - stride[MU];         \
    cx<double> u[9], p[12], h[6], g[6];                                                 \
    _Pragma("unroll") for (int e = 0; e < 9; e++) u[e] = ldc(U + (s * 4 + MU) * 9 + e); \
    _Pragma("unroll") for (int c = 0; c < 12; c++) p[c] = ldc(in + fw * 12 + c);        \
    project<MU, 1>(p, h);                                                               \
    su3_mul<0>(u, h, g);                                                                \
    reconstruct<MU, 1>(g, acc);                                                         \
    _Pragma("unroll") for (int e = 0; e < 9; e++) u[e] = ldc(U + (bw * 4 + MU) * 9 + e);\
    _Pragma("unroll") for (int c = 0; c < 12; c++) p[c] = ldc(in + bw * 12 + c);        \
    project<MU, -1>(p, h);                                                              \
    su3_mul<1>(u, h, g);                                                                \
    reconstruct<MU, -1>(g, acc);                                                        \
  }
  CANON_DIR(0)
  CANON_DIR(1)
  CANON_DIR(2)
  CANON_DIR(3)
#undef CANON_DIR
#pragma unroll
  for (int c = 0; c < 12; c++) {
    cx<double> p = ldc(in + s * 12 + c);
    stc(out + s * 12 + c, cx<double>{diag * p.re - 0.5 * acc[c].re, diag * p.im - 0.5 * acc[c].im});
  }
}

int wilson_canonical(const Geom &g, const double *U, double m, const double *in, double *out, hipStream_t st) {
  dim3 grid((unsigned)((g.V + 255) / 256));
  hipLaunchKernelGGL(k_wilson_canon, grid, dim3(256), 0, st, (const double2 *)U, (const double2 *)in, (double2 *)out,
                     g.L[0], g.L[1], g.L[2], g.L[3], g.V, 4.0 + m);
  WMG_HIP(hipGetLastError());
  return 0;
}

// ---------------------------------------------------------------- layouts
template <class TL> __global__ void k_links_to_soa(const double2 *__restrict__ Uc, TL *__restrict__ Us, long V) {
  long s = blockIdx.x * 256L + threadIdx.x;
  if (s >= V) return;
  for (int mu = 0; mu < 4; mu++)
    for (int e = 0; e < 9; e++) {
      double2 v = Uc[(s * 4 + mu) * 9 + e];
      TL *d = Us + (size_t)(mu * 9 + e) * V + s;
      if constexpr (sizeof(TL) == 16) *d = v;
      else if constexpr (sizeof(TL) == 8) *d = make_float2((float)v.x, (float)v.y);
      else *d = __floats2half2_rn((float)v.x, (float)v.y);
    }
}

int links_to_soa(const Geom &g, const double *Ucanon, int lprec, void *Usoa, hipStream_t st) {
  dim3 grid((unsigned)((g.V + 255) / 256));
  if (lprec == P64)
    hipLaunchKernelGGL((k_links_to_soa<double2>), grid, dim3(256), 0, st, (const double2 *)Ucanon, (double2 *)Usoa, g.V);
  else if (lprec == P32)
    hipLaunchKernelGGL((k_links_to_soa<float2>), grid, dim3(256), 0, st, (const double2 *)Ucanon, (float2 *)Usoa, g.V);
  else
    hipLaunchKernelGGL((k_links_to_soa<__half2>), grid, dim3(256), 0, st, (const double2 *)Ucanon, (__half2 *)Usoa, g.V);
  WMG_HIP(hipGetLastError());
  return 0;
}

__global__ void k_spinor_to_soa(const double2 *__restrict__ c, double2 *__restrict__ s, long V) {
  long i = blockIdx.x * 256L + threadIdx.x;
  int r = blockIdx.y;
  if (i >= V) return;
  for (int k = 0; k < 12; k++) s[((size_t)r * 12 + k) * V + i] = c[((size_t)r * V + i) * 12 + k];
}
__global__ void k_spinor_from_soa(const double2 *__restrict__ s, double2 *__restrict__ c, long V) {
  long i = blockIdx.x * 256L + threadIdx.x;
  int r = blockIdx.y;
  if (i >= V) return;
  for (int k = 0; k < 12; k++) c[((size_t)r * V + i) * 12 + k] = s[((size_t)r * 12 + k) * V + i];
}

int spinor_to_soa(const Geom &g, const double *canon, double2 *soa, int nrhs, hipStream_t st) {
  dim3 grid((unsigned)((g.V + 255) / 256), nrhs);
  hipLaunchKernelGGL(k_spinor_to_soa, grid, dim3(256), 0, st, (const double2 *)canon, soa, g.V);
  WMG_HIP(hipGetLastError());
  return 0;
}
int spinor_from_soa(const Geom &g, const double2 *soa, double *canon, int nrhs, hipStream_t st) {
  dim3 grid((unsigned)((g.V + 255) / 256), nrhs);
  hipLaunchKernelGGL(k_spinor_from_soa, grid, dim3(256), 0, st, soa, (double2 *)canon, g.V);
  WMG_HIP(hipGetLastError());
  return 0;
}

}  // namespace wmg
