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
// addresses.  A workgroup first copies the spinors of its own 256-site tile
// into LDS with one burst of coalesced loads; every hop whose neighbour lies
// in the tile (and the diagonal term) then reads LDS, and only neighbours in
// other tiles go to L2.  Reuse across tiles is left to L2/MALL, with
// workgroups mapped so that each XCD sweeps one contiguous range of sites.
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

// one colour of the projection: h0 = p0 - S (A p_down)_0, h1 = p1 - S (A p_down)_1
template <int MU, int S, class R> __device__ __forceinline__ void proj_pair(const cx<R> p[4], cx<R> &h0, cx<R> &h1) {
  cx<R> a0, a1;
  if (MU == 0) { a0 = times_mi(p[3]); a1 = times_mi(p[2]); }
  if (MU == 1) { a0 = neg(p[3]); a1 = p[2]; }
  if (MU == 2) { a0 = times_mi(p[2]); a1 = times_i(p[3]); }
  if (MU == 3) { a0 = p[2]; a1 = p[3]; }
  if (S > 0) { h0 = p[0] - a0; h1 = p[1] - a1; }
  else { h0 = p[0] + a0; h1 = p[1] + a1; }
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

// ---------------------------------------------------------------- work order
// Each XCD has its own 4 MB L2 and receives workgroups round-robin.  The
// lattice is cut into slabs (y and z split into ny x nz pieces, a multiple of
// 8 of them when possible) whose cross-section at fixed t is small.  Tiles
// of 256 sites are numbered slab by slab, inside a slab x fastest and t
// slowest, and XCD k takes the k-th contiguous eighth of that sequence: it
// sweeps its slabs in t order, so the previous and next t-slices of a site
// (and its y and z neighbours inside the slab) are in that XCD's L2 when
// they are needed.
struct SweepMap {
  int ny, nz;     // slab split of y and z
  int dy, dz;     // slab extents
  long vd;        // sites per slab
  long td;        // tiles per slab
  long per_xcd;   // tiles per XCD
  long nblocks;   // grid size (multiple of 8)
};

static SweepMap make_sweep(const int L[4], int bytes_per_site) {
  // among splits whose t-slice takes at most ~1 MB of L2, the one with the
  // smallest y/z face fraction (neighbours outside the slab); the largest
  // cross-section breaks ties.  If none fits, the smallest cross-section.
  const long budget = 1L << 20;
  SweepMap best{};
  best.ny = best.nz = 1;
  bool have = false, bfits = false;
  double bface = 0;
  long bcs = 0;
  for (int ny = 1; ny <= L[1]; ny++) {
    if (L[1] % ny) continue;
    for (int nz = 1; nz <= L[2]; nz++) {
      if (L[2] % nz || (ny * nz) % NXCD) continue;
      int dy = L[1] / ny, dz = L[2] / nz;
      long cs = (long)L[0] * dy * dz;
      bool fits = cs * bytes_per_site <= budget;
      double face = (dy < L[1] ? 1.0 / dy : 0.0) + (dz < L[2] ? 1.0 / dz : 0.0);
      bool better;
      if (!have) better = true;
      else if (fits != bfits) better = fits;
      else if (fits) better = face < bface - 1e-12 || (face < bface + 1e-12 && cs > bcs);
      else better = cs < bcs;
      if (better) {
        have = true;
        bfits = fits;
        bface = face;
        bcs = cs;
        best.ny = ny;
        best.nz = nz;
      }
    }
  }
  best.dy = L[1] / best.ny;
  best.dz = L[2] / best.nz;
  best.vd = (long)L[0] * best.dy * best.dz * L[3];
  best.td = (best.vd + 255) / 256;
  long ntile = (long)best.ny * best.nz * best.td;
  best.per_xcd = (ntile + NXCD - 1) / NXCD;
  best.nblocks = best.per_xcd * NXCD;
  return best;
}

// site handled by (workgroup b, thread t); false for padding slots
__device__ __forceinline__ bool sweep_site(const SweepMap &sm, const int L[4], long b, int t, int x[4], long &s) {
  long g = (b % NXCD) * sm.per_xcd + b / NXCD;  // tile in slab-major order
  long slab = g / sm.td;
  if (slab >= (long)sm.ny * sm.nz) return false;
  long q = (g % sm.td) * 256 + t;
  if (q >= sm.vd) return false;
  int iy = (int)(slab % sm.ny), iz = (int)(slab / sm.ny);
  x[0] = (int)(q % L[0]);
  q /= L[0];
  x[1] = (int)(q % sm.dy) + iy * sm.dy;
  q /= sm.dy;
  x[2] = (int)(q % sm.dz) + iz * sm.dz;
  x[3] = (int)(q / sm.dz);
  s = site_index(L, x);
  return true;
}

// ---------------------------------------------------------------- SoA
// Optional fusions for the smoother: bsub != nullptr gives out = bsub - D in
// (residual); RED != 0 also reduces <out, in> and |out|^2 over the
// workgroup into red[(rhs * gridDim.x + block) * 3 + 0..2] for a
// fixed-order finalisation by k_dslash_red_finalize.
template <class TL, class TS, class TO, int RT, int RED>
__global__ void __launch_bounds__(256) k_wilson_soa(const TL *__restrict__ U, const TS *__restrict__ in,
                                                   TO *__restrict__ out, int L0, int L1, int L2, int L3, long V,
                                                   float diagf, double diagd, int nrhs, SweepMap sm, long Vs,
                                                   const TS *__restrict__ bsub, const double *__restrict__ bnrm2,
                                                   int bstride, double *__restrict__ red, int inner,
                                                   float2 *__restrict__ out32) {
  using R = typename store_traits<TS>::real;
  const R diag = sizeof(R) == 8 ? (R)diagd : (R)diagf;
  // one sweep over the lattice per tile of RT right-hand sides (grid.y)
  const int L[4] = {L0, L1, L2, L3};
  int x[4];
  long s = 0;
  // site-tile workgroup index tb and first rhs r0: grid (tiles, rhs tiles),
  // or with `inner` one dimension in which each XCD (blockIdx % 8) takes the
  // rhs tiles of its site tiles consecutively
  long tb = blockIdx.x;
  int r0 = blockIdx.y * RT;
  if (inner) {
    const int nrt = (nrhs + RT - 1) / RT;
    const long q = (long)blockIdx.x / NXCD;
    tb = (q / nrt) * NXCD + blockIdx.x % NXCD;
    r0 = (int)(q % nrt) * RT;
  }
  const bool valid = sweep_site(sm, L, tb, threadIdx.x, x, s);
  // the tile's own spinors, [t][c][thread] (sized for the right-hand sides
  // this launch has, at most RT)
  extern __shared__ unsigned char dsm[];
  TS *Sh = (TS *)dsm;
  if (valid) {
#pragma unroll
    for (int t = 0; t < RT; t++)
      if (r0 + t < nrhs)
#pragma unroll
        for (int c = 0; c < 12; c++) Sh[(t * 12 + c) * 256 + threadIdx.x] = in[((size_t)(r0 + t) * 12 + c) * Vs + s];
  }
  __syncthreads();
  // tile-local slot of a neighbour site, -1 when it lies in another tile
  const long gtile = (tb % NXCD) * sm.per_xcd + tb / NXCD;
  const long ttile = gtile % sm.td, slab = gtile / sm.td;
  const int iy = (int)(slab % sm.ny), iz = (int)(slab / sm.ny);
  auto local_of = [&](const int y[4]) -> int {
    int ly = y[1] - iy * sm.dy, lz = y[2] - iz * sm.dz;
    if (ly < 0 || ly >= sm.dy || lz < 0 || lz >= sm.dz) return -1;
    long q = y[0] + (long)L0 * (ly + (long)sm.dy * (lz + (long)sm.dz * y[3]));
    return q / 256 == ttile ? (int)(q % 256) : -1;
  };
  double rs[RT][3];
#pragma unroll
  for (int t = 0; t < RT; t++) rs[t][0] = rs[t][1] = rs[t][2] = 0.0;
  if (valid) {
  long stride[4] = {1, (long)L0, (long)L0 * L1, (long)L0 * L1 * L2};
  cx<R> acc[RT][12];
#pragma unroll
  for (int t = 0; t < RT; t++)
#pragma unroll
    for (int c = 0; c < 12; c++) acc[t][c] = czero<R>();

  auto load_link = [&](int mu, long site, cx<R> u[9]) {
#pragma unroll
    for (int e = 0; e < 9; e++) {
      auto v = ldc(U + ((size_t)(mu * 9 + e)) * Vs + site);
      u[e] = {(R)v.re, (R)v.im};
    }
  };
  // half spinor of the neighbour, projected colour by colour straight from
  // the loads, then the link applied row by row (few live registers)
  auto hop_half = [&](int r, long site, int loc, auto proj, cx<R> h[6]) {
#pragma unroll
    for (int c = 0; c < 3; c++) {
      cx<R> p4[4];
#pragma unroll
      for (int sp = 0; sp < 4; sp++) {
        auto v = loc >= 0 ? ldc(Sh + ((r - r0) * 12 + sp * 3 + c) * 256 + loc)
                          : ldc(in + ((size_t)r * 12 + sp * 3 + c) * Vs + site);
        p4[sp] = {(R)v.re, (R)v.im};
      }
      proj(p4, h[c], h[3 + c]);
    }
  };
#define WILSON_DIR(MU)                                                                         \
  {                                                                                            \
    long fw = x[MU] == L[MU] - 1 ? s - (long)(L[MU] - 1) * stride[MU] : s + stride[MU];        \
    long bw = x[MU] == 0 ? s + (long)(L[MU] - 1) * stride[MU] : s - stride[MU];                \
    int yf[4] = {x[0], x[1], x[2], x[3]}, yb[4] = {x[0], x[1], x[2], x[3]};                    \
    yf[MU] = x[MU] == L[MU] - 1 ? 0 : x[MU] + 1;                                               \
    yb[MU] = x[MU] == 0 ? L[MU] - 1 : x[MU] - 1;                                               \
    const int lf = local_of(yf), lb = local_of(yb);                                            \
    cx<R> u[9], h[6], g[6];                                                                    \
    load_link(MU, s, u);                                                                       \
    _Pragma("unroll") for (int t = 0; t < RT; t++) {                                           \
      if (r0 + t < nrhs) {                                                                     \
        hop_half(r0 + t, fw, lf, proj_pair<MU, 1, R>, h);                                          \
        su3_mul<0>(u, h, g);                                                                   \
        reconstruct<MU, 1>(g, acc[t]);                                                         \
      }                                                                                        \
    }                                                                                          \
    load_link(MU, bw, u);                                                                      \
    _Pragma("unroll") for (int t = 0; t < RT; t++) {                                           \
      if (r0 + t < nrhs) {                                                                     \
        hop_half(r0 + t, bw, lb, proj_pair<MU, -1, R>, h);                                         \
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
#pragma unroll
    for (int c = 0; c < 12; c++) {
      auto v = ldc(Sh + (t * 12 + c) * 256 + threadIdx.x);
      p[c] = {(R)v.re, (R)v.im};
    }
#pragma unroll
    for (int c = 0; c < 12; c++) {
      cx<R> o = {diag * p[c].re - R(0.5) * acc[t][c].re, diag * p[c].im - R(0.5) * acc[t][c].im};
      if (bsub) {
        auto bv = ldc(bsub + ((size_t)(r0 + t) * 12 + c) * Vs + s);
        R bs = R(1);
        if (bnrm2) {
          double q = bnrm2[(size_t)(r0 + t) * bstride];
          bs = q > 0 ? (R)(1.0 / sqrt(q)) : R(0);
        }
        o = cx<R>{bs * (R)bv.re - o.re, bs * (R)bv.im - o.im};
      }
      stc(out + ((size_t)(r0 + t) * 12 + c) * Vs + s, o);
      if (out32) stc(out32 + ((size_t)(r0 + t) * 12 + c) * Vs + s, o);
      if (RED) o = as_stored(out, o);
      if (RED) {
        rs[t][0] += (double)o.re * p[c].re + (double)o.im * p[c].im;
        rs[t][1] += (double)o.re * p[c].im - (double)o.im * p[c].re;
        rs[t][2] += (double)o.re * o.re + (double)o.im * o.im;
      }
    }
  }
  }  // valid
  if (RED) {
    __shared__ double sh[RT][3][4];
    int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int t = 0; t < RT; t++)
#pragma unroll
      for (int q = 0; q < 3; q++) {
        double v = rs[t][q];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
        if (lane == 0) sh[t][q][wv] = v;
      }
    __syncthreads();
    if (threadIdx.x < RT * 3) {
      int t = threadIdx.x / 3, q = threadIdx.x % 3;
      if (r0 + t < nrhs)
        red[((size_t)(r0 + t) * sm.nblocks + tb) * 3 + q] = sh[t][q][0] + sh[t][q][1] + sh[t][q][2] + sh[t][q][3];
    }
  }
}

// out[rhs*stride + 0..2] = sum over blocks of red[(rhs*nblk + b)*3 + 0..2],
// summed in a fixed order (one workgroup per rhs)
__global__ void __launch_bounds__(256) k_dslash_red_finalize(const double *__restrict__ red, long nblk,
                                                            double *__restrict__ out, int stride) {
  int rhs = blockIdx.x;
  double v[3] = {0, 0, 0};
  for (long b = threadIdx.x; b < nblk; b += 256)
#pragma unroll
    for (int q = 0; q < 3; q++) v[q] += red[((size_t)rhs * nblk + b) * 3 + q];
  __shared__ double sh[3][4];
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < 3; q++) {
    double x = v[q];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
    if (lane == 0) sh[q][wv] = x;
  }
  __syncthreads();
  if (threadIdx.x < 3) out[(size_t)rhs * stride + threadIdx.x] = sh[threadIdx.x][0] + sh[threadIdx.x][1] +
                                                                   sh[threadIdx.x][2] + sh[threadIdx.x][3];
}

template <class TL, class TS, class TO = TS>
static void launch_soa(const Geom &g, const void *U, double m, const void *in, void *out, int nrhs, const void *bsub,
                       double *red, double *red_out, int red_stride, hipStream_t st, const double *bnrm2 = nullptr,
                       int bstride = 0, void *out32 = nullptr) {
  constexpr int RT = sizeof(TS) == 16 ? 1 : 2;
  const int nrt = (nrhs + RT - 1) / RT;
  // FP64 and FP32 links (288-576 B per site) would be re-read from HBM by
  // every rhs tile's sweep: the rhs tiles of one site tile then run back to
  // back on one XCD and share the links in its L2 (FP64, 28 rhs: 14.6 ->
  // 10.4 ms on 32^3x64).  FP16 links are cheap to re-read, and one sweep per
  // rhs tile keeps the spinor halo in L2.
  const int inner = sizeof(TL) >= 8 && nrt > 1;
  // bytes a site brings into L2 during one sweep: its links and RT spinors
  SweepMap sm = make_sweep(g.L, 36 * (int)sizeof(TL) + 24 * (int)sizeof(TS) / 2 * RT);
  dim3 grid = inner ? dim3((unsigned)(sm.nblocks * nrt)) : dim3((unsigned)sm.nblocks, nrt);
  const size_t lds = (size_t)(nrhs < RT ? nrhs : RT) * 12 * 256 * sizeof(TS);
  if (red) {
    hipLaunchKernelGGL((k_wilson_soa<TL, TS, TO, RT, 1>), grid, dim3(256), lds, st, (const TL *)U, (const TS *)in,
                       (TO *)out, g.L[0], g.L[1], g.L[2], g.L[3], g.V, (float)(4.0 + m), 4.0 + m, nrhs, sm, g.Vs,
                       (const TS *)bsub, bnrm2, bstride, red, inner, (float2 *)out32);
    hipLaunchKernelGGL(k_dslash_red_finalize, dim3(nrhs), dim3(256), 0, st, red, (long)sm.nblocks, red_out,
                       red_stride);
  } else {
    hipLaunchKernelGGL((k_wilson_soa<TL, TS, TO, RT, 0>), grid, dim3(256), lds, st, (const TL *)U, (const TS *)in,
                       (TO *)out, g.L[0], g.L[1], g.L[2], g.L[3], g.V, (float)(4.0 + m), 4.0 + m, nrhs, sm, g.Vs,
                       (const TS *)bsub, bnrm2, bstride, (double *)nullptr, inner, (float2 *)out32);
  }
}

long wilson_red_blocks(const Geom &g) {
  // every (link, spinor) storage pair launch_soa instantiates
  const int bps[4] = {36 * 16 + 24 * 8, 36 * 8 + 24 * 4 * 2, 36 * 4 + 24 * 4 * 2, 36 * 4 + 24 * 2 * 2};
  long m = 0;
  for (int i = 0; i < 4; i++) {
    long nb = make_sweep(g.L, bps[i]).nblocks;
    m = nb > m ? nb : m;
  }
  return m;
}

int wilson_soa_fused(const Geom &g, int lprec, const void *U, int sprec, double m, const void *in, void *out, int nrhs,
                     const void *bsub, double *red, double *red_out, int red_stride, hipStream_t st, void *out32) {
  if (out32 && sprec != P64) return set_error(-1, "wilson_soa: FP32 copy of the output only for FP64 spinors");
  if (sprec == P64 && lprec == P64)
    launch_soa<double2, double2>(g, U, m, in, out, nrhs, bsub, red, red_out, red_stride, st, nullptr, 0, out32);
  else if (sprec == P32 && lprec == P32)
    launch_soa<float2, float2>(g, U, m, in, out, nrhs, bsub, red, red_out, red_stride, st);
  else if (sprec == P32 && lprec == P16)
    launch_soa<__half2, float2>(g, U, m, in, out, nrhs, bsub, red, red_out, red_stride, st);
  else return set_error(-1, "wilson_soa: unsupported precision pair link=%d spinor=%d", lprec, sprec);
  WMG_HIP(hipGetLastError());
  return 0;
}

int wilson_soa_h16(const Geom &g, const void *U16, int iprec, double m, const void *in, void *out, int nrhs,
                   const void *bsub, const double *bnrm2, int bstride, double *red, double *red_out, int red_stride,
                   hipStream_t st) {
  if (iprec == P32)
    launch_soa<__half2, float2, __half2>(g, U16, m, in, out, nrhs, bsub, red, red_out, red_stride, st, bnrm2, bstride);
  else if (iprec == P16 && !bsub)
    launch_soa<__half2, __half2, __half2>(g, U16, m, in, out, nrhs, nullptr, red, red_out, red_stride, st);
  else return set_error(-1, "wilson_soa_h16: input precision %d%s", iprec, bsub ? " with bsub" : "");
  WMG_HIP(hipGetLastError());
  return 0;
}

int wilson_soa(const Geom &g, int lprec, const void *U, int sprec, double m, const void *in, void *out, int nrhs,
               hipStream_t st) {
  return wilson_soa_fused(g, lprec, U, sprec, m, in, out, nrhs, nullptr, nullptr, nullptr, 0, st);
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
template <class TL>
__global__ void k_links_to_soa(const double2 *__restrict__ Uc, TL *__restrict__ Us, long V, long Vs) {
  long s = blockIdx.x * 256L + threadIdx.x;
  if (s >= V) return;
  for (int mu = 0; mu < 4; mu++)
    for (int e = 0; e < 9; e++) {
      double2 v = Uc[(s * 4 + mu) * 9 + e];
      TL *d = Us + (size_t)(mu * 9 + e) * Vs + s;
      if constexpr (sizeof(TL) == 16) *d = v;
      else if constexpr (sizeof(TL) == 8) *d = make_float2((float)v.x, (float)v.y);
      else *d = __floats2half2_rn((float)v.x, (float)v.y);
    }
}

int links_to_soa(const Geom &g, const double *Ucanon, int lprec, void *Usoa, hipStream_t st) {
  dim3 grid((unsigned)((g.V + 255) / 256));
  if (lprec == P64)
    hipLaunchKernelGGL((k_links_to_soa<double2>), grid, dim3(256), 0, st, (const double2 *)Ucanon, (double2 *)Usoa, g.V, g.Vs);
  else if (lprec == P32)
    hipLaunchKernelGGL((k_links_to_soa<float2>), grid, dim3(256), 0, st, (const double2 *)Ucanon, (float2 *)Usoa, g.V, g.Vs);
  else
    hipLaunchKernelGGL((k_links_to_soa<__half2>), grid, dim3(256), 0, st, (const double2 *)Ucanon, (__half2 *)Usoa, g.V, g.Vs);
  WMG_HIP(hipGetLastError());
  return 0;
}

__global__ void k_spinor_to_soa(const double2 *__restrict__ c, double2 *__restrict__ s, long V, long Vs) {
  long i = blockIdx.x * 256L + threadIdx.x;
  int r = blockIdx.y;
  if (i >= V) return;
  for (int k = 0; k < 12; k++) s[((size_t)r * 12 + k) * Vs + i] = c[((size_t)r * V + i) * 12 + k];
}
__global__ void k_spinor_from_soa(const double2 *__restrict__ s, double2 *__restrict__ c, long V, long Vs) {
  long i = blockIdx.x * 256L + threadIdx.x;
  int r = blockIdx.y;
  if (i >= V) return;
  for (int k = 0; k < 12; k++) c[((size_t)r * V + i) * 12 + k] = s[((size_t)r * 12 + k) * Vs + i];
}

int spinor_to_soa(const Geom &g, const double *canon, double2 *soa, int nrhs, hipStream_t st) {
  dim3 grid((unsigned)((g.V + 255) / 256), nrhs);
  hipLaunchKernelGGL(k_spinor_to_soa, grid, dim3(256), 0, st, (const double2 *)canon, soa, g.V, g.Vs);
  WMG_HIP(hipGetLastError());
  return 0;
}
int spinor_from_soa(const Geom &g, const double2 *soa, double *canon, int nrhs, hipStream_t st) {
  dim3 grid((unsigned)((g.V + 255) / 256), nrhs);
  hipLaunchKernelGGL(k_spinor_from_soa, grid, dim3(256), 0, st, soa, (double2 *)canon, g.V, g.Vs);
  WMG_HIP(hipGetLastError());
  return 0;
}

}  // namespace wmg
