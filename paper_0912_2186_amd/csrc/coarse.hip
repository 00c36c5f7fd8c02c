// Coarse operator of the adaptive multigrid (arXiv:0912.2186, Sec. 2-3 and
// Sec. 4's dense N_nu x N_nu coarse-link algebra).
//
// Build: D_hat = P^dag D P (Galerkin, R = P^dag) stored as a 9-point stencil
// with dense n x n complex blocks, n = 2 N_nu:
//   out(xh) = X(xh) in(xh) + sum_mu [ Y_{+mu}(xh) in(xh+mu) + Y_{-mu}(xh) in(xh-mu) ].
// For coarse column (chi_c, alpha) the fine vector v = Pi_chi_c P[alpha]
// (all aggregates at once) is hit by the fine operator split by hop class
// (0: diagonal + hops inside the target's aggregate; 1+mu / 5+mu: hops
// across the +mu / -mu face) and each class is restricted on the target
// aggregate.  Classes are kept by hop direction, so forward and backward
// links stay apart even where a coarse extent is 1 or 2.
//
// Internal link layout (for coalesced apply): [Vc][9][col][row], i.e. the
// element (row, col) of block d of site xh sits at ((xh*9+d)*n + col)*n + row.
#include <mutex>

#include "wmg_internal.h"

namespace wmg {

static constexpr int TB = 256;

struct CGeom {
  int L[4], b[4], Lc[4];
  long V, Vc;
  long Vs;  // fine-lattice site stride of the links
  int bs, dof, nv;
  int ns;   // parts of the fine site's 12 components: 2 chiralities or 4 spins
  // storage of the built blocks: coarse index (part, alpha) at part * nld +
  // alpha of a block with leading dimension ldn (nld = nv, ldn = ns * nv for
  // the compact layout); columns computed: alpha = al0 .. al0 + gridDim.y/ns - 1
  int nld, ldn, al0;
};

__device__ __forceinline__ long cg_block_site(const CGeom &g, long xh, int k, int x[4]) {
  int xc[4];
  site_coords(g.Lc, xh, xc);
  int w0 = k % g.b[0], r = k / g.b[0];
  int w1 = r % g.b[1]; r /= g.b[1];
  int w2 = r % g.b[2]; int w3 = r / g.b[2];
  x[0] = xc[0] * g.b[0] + w0;
  x[1] = xc[1] * g.b[1] + w1;
  x[2] = xc[2] * g.b[2] + w2;
  x[3] = xc[3] * g.b[3] + w3;
  return site_index(g.L, x);
}

// (coarse site, element-in-block k) of a fine site given its coordinates
__device__ __forceinline__ void cg_locate(const CGeom &g, const int x[4], long &xh, int &k) {
  int xc[4], w[4];
  for (int i = 0; i < 4; i++) {
    xc[i] = x[i] / g.b[i];
    w[i] = x[i] % g.b[i];
  }
  xh = site_index(g.Lc, xc);
  k = w[0] + g.b[0] * (w[1] + g.b[1] * (w[2] + g.b[2] * w[3]));
}

template <int NV>
__device__ __forceinline__ void cg_wsum(cx<double> v[NV], double *sh, double *out) {
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < NV; j++) {
    double a = v[j].re, b = v[j].im;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      a += __shfl_down(a, o, 64);
      b += __shfl_down(b, o, 64);
    }
    if (lane == 0) {
      sh[w * 2 * NV + 2 * j] = a;
      sh[w * 2 * NV + 2 * j + 1] = b;
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * NV) {
    double x = 0;
    for (int q = 0; q < TB / 64; q++) x += sh[q * 2 * NV + threadIdx.x];
    out[threadIdx.x] = x;
  }
  __syncthreads();
}

// Wilson hop (Eq. 2.2, gauge-covariant placement) written out with the full
// gamma matrices: forward -1/2 (1-gamma_mu) U_mu(x) v(x+mu), backward
// -1/2 (1+gamma_mu) U_mu(x-mu)^dag v(x-mu).
__constant__ double2 c_gamma[4][4][4];

__device__ __forceinline__ void wilson_hop(const double2 *U, long V, long s, long t, int mu, int sg,
                                           const cx<double> in[12], cx<double> out[12]) {
  cx<double> uv[4][3];
  long ls = sg > 0 ? s : t;
  for (int sp = 0; sp < 4; sp++)
    for (int a = 0; a < 3; a++) {
      cx<double> acc = czero<double>();
      for (int b = 0; b < 3; b++) {
        if (sg > 0) acc = cfma(ldc(U + (size_t)(mu * 9 + 3 * a + b) * V + ls), in[3 * sp + b], acc);
        else acc = cfmac(ldc(U + (size_t)(mu * 9 + 3 * b + a) * V + ls), in[3 * sp + b], acc);
      }
      uv[sp][a] = acc;
    }
  for (int i = 0; i < 4; i++)
    for (int a = 0; a < 3; a++) {
      cx<double> acc = czero<double>();
      for (int j = 0; j < 4; j++) {
        double2 gg = c_gamma[mu][i][j];
        cx<double> g = {(sg > 0 ? -gg.x : gg.x) + (i == j ? 1.0 : 0.0), sg > 0 ? -gg.y : gg.y};  // 1 -+ gamma
        acc = cfma(g, uv[j][a], acc);
      }
      out[3 * i + a] = out[3 * i + a] + cx<double>{-0.5 * acc.re, -0.5 * acc.im};
    }
}

// One workgroup per (coarse site xh, column); fine Wilson level, one thread
// per fine site of the aggregate (bs <= 256).  NS parts per site (2
// chiralities or 4 spins), hc = 12 / NS components each.
template <int NS>
__global__ void __launch_bounds__(TB) k_build_wilson(CGeom g, const double2 *__restrict__ U, double m,
                                                    const double2 *__restrict__ P, double2 *__restrict__ Yc) {
  long xh = blockIdx.x;
  constexpr int hc = 12 / NS;
  const int nv = g.nv, n = NS * nv;
  const int nal = gridDim.y / NS;
  const int chic = blockIdx.y / nal, al = g.al0 + blockIdx.y % nal;
  const int colS = chic * g.nld + al;
  __shared__ double sh[4 * 2 * 16];
  __shared__ double red[2 * 16];
  int k = threadIdx.x;
  bool act = k < g.bs;
  int x[4] = {0, 0, 0, 0};
  long s = 0;
  if (act) s = cg_block_site(g, xh, k, x);
  const long E = (long)g.bs * 12;
  // v(site) = part chic (chirality or spin) of P[al] at that site
  auto loadv = [&](const int y[4], cx<double> v[12]) {
    long yh;
    int ky;
    cg_locate(g, y, yh, ky);
    for (int c = 0; c < 12; c++) {
      v[c] = (c / hc == chic) ? ldc(P + ((size_t)al * g.Vc + yh) * E + (size_t)c * g.bs + ky) : czero<double>();
    }
  };
  for (int d = 0; d < 9; d++) {
    cx<double> w[12];
    for (int c = 0; c < 12; c++) w[c] = czero<double>();
    // only sites on the block face crossed by direction d contribute to d > 0
    bool nz = act && d == 0;
    if (act) {
      if (d == 0) {
        cx<double> v[12];
        loadv(x, v);
        for (int c = 0; c < 12; c++) w[c] = (4.0 + m) * v[c];
      }
      for (int mu = 0; mu < 4; mu++)
        for (int sg = -1; sg <= 1; sg += 2) {
          bool cross = sg > 0 ? (x[mu] % g.b[mu] == g.b[mu] - 1) : (x[mu] % g.b[mu] == 0);
          int cls = cross ? (sg > 0 ? 1 + mu : 5 + mu) : 0;
          if (cls != d) continue;
          nz = true;
          int y[4] = {x[0], x[1], x[2], x[3]};
          y[mu] = (y[mu] + sg + g.L[mu]) % g.L[mu];
          cx<double> v[12];
          loadv(y, v);
          long t = site_index(g.L, y);
          wilson_hop(U, g.Vs, s, t, mu, sg, v, w);
        }
    }
    // restrict w onto rows (chi_r, beta), 16 rows at a time
    for (int r0 = 0; r0 < n; r0 += 16) {
      cx<double> acc[16];
#pragma unroll
      for (int j = 0; j < 16; j++) {
        acc[j] = czero<double>();
        int row = r0 + j;
        if (nz && row < n) {
          int chir = row / nv, be = row % nv;
          for (int c = chir * hc; c < chir * hc + hc; c++)
            acc[j] = cfmac(ldc(P + ((size_t)be * g.Vc + xh) * E + (size_t)c * g.bs + k), w[c], acc[j]);
        }
      }
      cg_wsum<16>(acc, sh, red);
      if (threadIdx.x < 16 && r0 + (int)threadIdx.x < n) {
        const int row = r0 + threadIdx.x;
        const int rowS = (row / nv) * g.nld + row % nv;
        Yc[(((size_t)xh * 9 + d) * g.ldn + colS) * g.ldn + rowS] =
            make_double2(red[2 * threadIdx.x], red[2 * threadIdx.x + 1]);
      }
      __syncthreads();
    }
  }
}

// Coarse level: the operator being coarsened is itself a 9-point stencil
// with dof f (internal layout).  One thread per aggregate element (k, c).
template <int EPT>
__global__ void __launch_bounds__(TB) k_build_coarse(CGeom g, const double2 *__restrict__ Yf,
                                                    const double2 *__restrict__ P, double2 *__restrict__ Yc) {
  long xh = blockIdx.x;
  int nv = g.nv, n = 2 * nv, f = g.dof, h = f / 2;
  const int nal = gridDim.y / 2;
  const int chic = blockIdx.y / nal, al = g.al0 + blockIdx.y % nal;
  const int colS = chic * g.nld + al;
  const long E = (long)g.bs * f;
  __shared__ double sh[4 * 2 * 16];
  __shared__ double red[2 * 16];
  for (int d = 0; d < 9; d++) {
    cx<double> w[EPT];
    int kk[EPT], cc[EPT];
    for (int q = 0; q < EPT; q++) {
      w[q] = czero<double>();
      kk[q] = -1;
      int e = threadIdx.x + q * TB;
      if (e >= E) continue;
      int k = e / f, c = e % f;
      kk[q] = k;
      cc[q] = c;
      int x[4];
      long s = cg_block_site(g, xh, k, x);
      // hops of the fine stencil at x: d' = 0 local, 1+mu, 5+mu
      for (int dd = 0; dd < 9; dd++) {
        int cls;
        int y[4] = {x[0], x[1], x[2], x[3]};
        if (dd == 0) cls = 0;
        else {
          int mu = (dd - 1) % 4, sg = dd <= 4 ? 1 : -1;
          bool cross = sg > 0 ? (x[mu] % g.b[mu] == g.b[mu] - 1) : (x[mu] % g.b[mu] == 0);
          cls = cross ? dd : 0;
          y[mu] = (y[mu] + sg + g.L[mu]) % g.L[mu];
        }
        if (cls != d) continue;
        long yh;
        int ky;
        cg_locate(g, y, yh, ky);
        // sum_c' Yf[s][dd][c][c'] v(y)[c'], v = chirality chic part of P[al]
        for (int c2 = chic * h; c2 < chic * h + h; c2++) {
          cx<double> yv = ldc(Yf + (((size_t)s * 9 + dd) * f + c2) * f + c);
          cx<double> pv = ldc(P + ((size_t)al * g.Vc + yh) * E + (size_t)ky * f + c2);
          w[q] = cfma(yv, pv, w[q]);
        }
      }
    }
    for (int r0 = 0; r0 < n; r0 += 16) {
      cx<double> acc[16];
#pragma unroll
      for (int j = 0; j < 16; j++) {
        acc[j] = czero<double>();
        int row = r0 + j;
        if (row < n) {
          int chir = row / nv, be = row % nv;
          for (int q = 0; q < EPT; q++) {
            if (kk[q] < 0 || cc[q] / h != chir) continue;
            int e = threadIdx.x + q * TB;
            acc[j] = cfmac(ldc(P + ((size_t)be * g.Vc + xh) * E + e), w[q], acc[j]);
          }
        }
      }
      cg_wsum<16>(acc, sh, red);
      if (threadIdx.x < 16 && r0 + (int)threadIdx.x < n) {
        int row = r0 + threadIdx.x;
        const int rowS = (row / nv) * g.nld + row % nv;
        Yc[(((size_t)xh * 9 + d) * g.ldn + colS) * g.ldn + rowS] =
            make_double2(red[2 * threadIdx.x], red[2 * threadIdx.x + 1]);
      }
      __syncthreads();
    }
  }
}

// The gamma table is uploaded once per process (std::call_once: concurrent
// setups of a batch may reach this together).
static std::once_flag gamma_once;
static int gamma_status = 0;
static int upload_gamma_once() {  // chiral basis: gamma_k = [[0, -i sigma_k], [i sigma_k, 0]], gamma_4 = [[0,1],[1,0]]
  double2 G[4][4][4];
  for (int mu = 0; mu < 4; mu++)
    for (int i = 0; i < 4; i++)
      for (int j = 0; j < 4; j++) G[mu][i][j] = make_double2(0, 0);
  // sigma matrices
  const double s_re[3][2][2] = {{{0, 1}, {1, 0}}, {{0, 0}, {0, 0}}, {{1, 0}, {0, -1}}};
  const double s_im[3][2][2] = {{{0, 0}, {0, 0}}, {{0, -1}, {1, 0}}, {{0, 0}, {0, 0}}};
  for (int k = 0; k < 3; k++)
    for (int i = 0; i < 2; i++)
      for (int j = 0; j < 2; j++) {
        // upper-right: -i sigma ; lower-left: +i sigma ;  i*(a+ib) = -b + ia
        G[k][i][2 + j] = make_double2(s_im[k][i][j], -s_re[k][i][j]);
        G[k][2 + i][j] = make_double2(-s_im[k][i][j], s_re[k][i][j]);
      }
  for (int i = 0; i < 2; i++) {
    G[3][i][2 + i] = make_double2(1, 0);
    G[3][2 + i][i] = make_double2(1, 0);
  }
  WMG_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_gamma), G, sizeof(G)));
  // complete before any kernel of a (non-blocking) context stream reads it
  WMG_HIP(hipDeviceSynchronize());
  return 0;
}
static int upload_gamma() {
  std::call_once(gamma_once, [] { gamma_status = upload_gamma_once(); });
  return gamma_status;
}

// columns alpha = al0 .. al0 + nal - 1 of every part, all ns * nv rows, into
// blocks of leading dimension ns * nld
static int build_cols(const Geom &gf, int fine_kind, int dof, const void *U64soa, double m, const double2 *Yf,
                      const int b[4], int nv, int nld, int al0, int nal, const double2 *P, double2 *Yc, hipStream_t st,
                      int ns) {
  CGeom g;
  for (int i = 0; i < 4; i++) {
    g.L[i] = gf.L[i];
    g.b[i] = b[i];
    g.Lc[i] = gf.L[i] / b[i];
  }
  g.V = gf.V;
  g.Vs = gf.Vs;
  g.Vc = (long)g.Lc[0] * g.Lc[1] * g.Lc[2] * g.Lc[3];
  g.bs = b[0] * b[1] * b[2] * b[3];
  g.dof = fine_kind == 0 ? 12 : dof;
  g.nv = nv;
  g.ns = fine_kind == 0 ? ns : 2;
  g.nld = nld;
  g.ldn = g.ns * nld;
  g.al0 = al0;
  if (g.ns != 2 && g.ns != 4) return set_error(-1, "coarse_build: %d parts", g.ns);
  if (nv > nld || al0 < 0 || nal < 1 || al0 + nal > nv) return set_error(-1, "coarse_build: columns out of range");
  dim3 grid((unsigned)g.Vc, g.ns * nal);
  if (fine_kind == 0) {
    if (g.bs > TB) return set_error(-1, "coarse_build: aggregate of %d sites > %d", g.bs, TB);
    int rc = upload_gamma();
    if (rc) return rc;
    if (g.ns == 4) hipLaunchKernelGGL(k_build_wilson<4>, grid, dim3(TB), 0, st, g, (const double2 *)U64soa, m, P, Yc);
    else hipLaunchKernelGGL(k_build_wilson<2>, grid, dim3(TB), 0, st, g, (const double2 *)U64soa, m, P, Yc);
  } else {
    long E = (long)g.bs * g.dof;
    int ept = (int)((E + TB - 1) / TB);
    if (ept <= 4) hipLaunchKernelGGL((k_build_coarse<4>), grid, dim3(TB), 0, st, g, Yf, P, Yc);
    else if (ept <= 8) hipLaunchKernelGGL((k_build_coarse<8>), grid, dim3(TB), 0, st, g, Yf, P, Yc);
    else if (ept <= 16) hipLaunchKernelGGL((k_build_coarse<16>), grid, dim3(TB), 0, st, g, Yf, P, Yc);
    else return set_error(-1, "coarse_build: aggregate too large (%ld elements)", E);
  }
  WMG_HIP(hipGetLastError());
  return 0;
}

int coarse_build(const Geom &gf, int fine_kind, int dof, const void *U64soa, double m, const double2 *Yf, const int b[4],
                 int nv, const double2 *P, double2 *Yc, double2 * /*work*/, hipStream_t st, int ns) {
  return build_cols(gf, fine_kind, dof, U64soa, m, Yf, b, nv, nv, 0, nv, P, Yc, st, ns);
}

// The rows of the newest vector from the columns just built, by the
// gamma_5-hermiticity of the coarse operator: sigma_3 D_hat sigma_3 =
// D_hat^dag (sigma_3 = +1 on the first half of the parts, -1 on the
// second), block by block D_hat(y, x) = sigma_3 D_hat(x, y)^dag sigma_3, i.e.
//   X(x)[i][j]        = s_i s_j conj(X(x)[j][i])
//   Y_{+mu}(x)[i][j]  = s_i s_j conj(Y_{-mu}(x+mu)[j][i])
//   Y_{-mu}(x)[i][j]  = s_i s_j conj(Y_{+mu}(x-mu)[j][i])
// for i a row of the newest vector (alpha = knew - 1) and j an older column.
// One thread per (coarse site, block, part of the new row, older column).
__global__ void k_mirror_new_rows(double2 *__restrict__ Y, int Lc0, int Lc1, int Lc2, int Lc3, long Vc, int ns,
                                  int nld, int knew) {
  const int nold = knew - 1;
  const long per = 9L * ns * ns * nold;
  const long i = blockIdx.x * 256L + threadIdx.x;
  if (nold < 1 || i >= Vc * per) return;
  const long xh = i / per;
  long r = i % per;
  const int d = (int)(r / ((long)ns * ns * nold));
  r %= (long)ns * ns * nold;
  const int chr = (int)(r / (ns * nold));
  r %= ns * nold;
  const int chj = (int)(r / nold), aj = (int)(r % nold);
  const int L[4] = {Lc0, Lc1, Lc2, Lc3};
  int x[4];
  site_coords(L, xh, x);
  int dp = 0;
  if (d >= 1) {
    const int mu = (d - 1) % 4, sg = d <= 4 ? 1 : -1;
    x[mu] = (x[mu] + sg + L[mu]) % L[mu];
    dp = sg > 0 ? 5 + mu : 1 + mu;
  }
  const long yh = site_index(L, x);
  const int ldn = ns * nld;
  const int rowS = chr * nld + nold, colS = chj * nld + aj;
  const double2 v = Y[(((size_t)yh * 9 + dp) * ldn + rowS) * ldn + colS];
  const double sgn = ((chr < ns / 2) == (chj < ns / 2)) ? 1.0 : -1.0;
  Y[(((size_t)xh * 9 + d) * ldn + colS) * ldn + rowS] = make_double2(sgn * v.x, -sgn * v.y);
}

// blocks of leading dimension ns * nld -> compact blocks of the first k
// vectors (n = ns * k)
__global__ void k_pack_blocks(const double2 *__restrict__ Ys, double2 *__restrict__ Yc, long Vc, int ns, int nld,
                              int k) {
  const int n = ns * k, ldn = ns * nld;
  const long i = blockIdx.x * 256L + threadIdx.x;
  if (i >= Vc * 9L * n * n) return;
  const long blk = i / ((long)n * n);
  const int e = (int)(i % ((long)n * n));
  const int c = e / n, rr = e % n;
  const int cS = (c / k) * nld + c % k, rS = (rr / k) * nld + rr % k;
  Yc[i] = Ys[(blk * ldn + cS) * ldn + rS];
}

int coarse_build_next(const Geom &gf, int fine_kind, int dof, const void *U64soa, double m, const double2 *Yf,
                      const int b[4], int k, int nld, const double2 *P, double2 *Ys, double2 *Yc, hipStream_t st,
                      int ns) {
  if (k < 1 || k > nld) return set_error(-1, "coarse_build_next: %d vectors of %d", k, nld);
  const int rc = build_cols(gf, fine_kind, dof, U64soa, m, Yf, b, k, nld, k - 1, 1, P, Ys, st, ns);
  if (rc) return rc;
  const int nsx = fine_kind == 0 ? ns : 2;
  int Lc[4];
  for (int i = 0; i < 4; i++) Lc[i] = gf.L[i] / b[i];
  const long Vc = (long)Lc[0] * Lc[1] * Lc[2] * Lc[3];
  if (k > 1) {
    const long nm = Vc * 9L * nsx * nsx * (k - 1);
    hipLaunchKernelGGL(k_mirror_new_rows, dim3((unsigned)((nm + 255) / 256)), dim3(256), 0, st, Ys, Lc[0], Lc[1],
                       Lc[2], Lc[3], Vc, nsx, nld, k);
    WMG_HIP(hipGetLastError());
  }
  const long np = Vc * 9L * nsx * k * nsx * k;
  hipLaunchKernelGGL(k_pack_blocks, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, Ys, Yc, Vc, nsx, nld, k);
  WMG_HIP(hipGetLastError());
  return 0;
}

// ------------------------------------------------------------ apply
// One wavefront per (coarse site, rhs): lane = output row.  The nine input
// vectors are staged in LDS (sigma_3 applied for the adjoint, which for a
// gamma_5-hermitian coarse operator is D_hat^dag = sigma_3 D_hat sigma_3).
template <class TY, class TV, int NMAX>
__global__ void __launch_bounds__(TB) k_coarse_apply(const TY *__restrict__ Y, const TV *__restrict__ in,
                                                    TV *__restrict__ out, int L0, int L1, int L2, int L3, long Vc, int n,
                                                    int dagger, int nrhs) {
  using R = typename store_traits<TV>::real;
  __shared__ cx<R> vin[TB / 64][9][NMAX];
  int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  long item = (long)blockIdx.x * (TB / 64) + wv;
  long xh = item % Vc;
  int r = (int)(item / Vc);
  bool act = r < nrhs;
  const int L[4] = {L0, L1, L2, L3};
  int x[4];
  site_coords(L, act ? xh : 0, x);
  long nb[9];
  nb[0] = xh;
  for (int mu = 0; mu < 4; mu++) {
    int y[4] = {x[0], x[1], x[2], x[3]};
    y[mu] = (x[mu] + 1) % L[mu];
    nb[1 + mu] = site_index(L, y);
    y[mu] = (x[mu] - 1 + L[mu]) % L[mu];
    nb[5 + mu] = site_index(L, y);
  }
  int h = n / 2;
  if (act)
    for (int d = 0; d < 9; d++)
      for (int c = lane; c < n; c += 64) {
        auto v = ldc(in + ((size_t)r * Vc + nb[d]) * n + c);
        cx<R> t = {(R)v.re, (R)v.im};
        vin[wv][d][c] = (dagger && c >= h) ? neg(t) : t;
      }
  __syncthreads();
  if (!act) return;
  for (int row = lane; row < n; row += 64) {
    cx<R> acc = czero<R>();
    for (int d = 0; d < 9; d++) {
      const TY *yb = Y + ((size_t)xh * 9 + d) * n * n + row;
      for (int c = 0; c < n; c++) {
        auto yv = ldc(yb + (size_t)c * n);
        acc = cfma(cx<R>{(R)yv.re, (R)yv.im}, vin[wv][d][c], acc);
      }
    }
    if (dagger && row >= h) acc = neg(acc);
    stc(out + ((size_t)r * Vc + xh) * n + row, acc);
  }
}

int coarse_apply(const Geom &gc, int n, int yprec, const void *Y, int vprec, const void *in, void *out, int dagger,
                 int nrhs, hipStream_t st) {
  long items = gc.V * nrhs;
  dim3 grid((unsigned)((items + TB / 64 - 1) / (TB / 64)));
  if (n > 128) return set_error(-1, "coarse_apply: n=%d > 128", n);
  if (yprec == P64 && vprec == P64)
    hipLaunchKernelGGL((k_coarse_apply<double2, double2, 128>), grid, dim3(TB), 0, st, (const double2 *)Y,
                       (const double2 *)in, (double2 *)out, gc.L[0], gc.L[1], gc.L[2], gc.L[3], gc.V, n, dagger, nrhs);
  else if (yprec == P32 && vprec == P32)
    hipLaunchKernelGGL((k_coarse_apply<float2, float2, 128>), grid, dim3(TB), 0, st, (const float2 *)Y,
                       (const float2 *)in, (float2 *)out, gc.L[0], gc.L[1], gc.L[2], gc.L[3], gc.V, n, dagger, nrhs);
  else
    return set_error(-1, "coarse_apply: unsupported precision pair %d %d", yprec, vprec);
  WMG_HIP(hipGetLastError());
  return 0;
}

__global__ void k_shift_diag(long Vc, int n, double2 *Y, double dm) {
  long i = blockIdx.x * (long)TB + threadIdx.x;
  if (i >= Vc * n) return;
  long xh = i / n;
  int r = (int)(i % n);
  double2 *p = Y + (((size_t)xh * 9 + 0) * n + r) * n + r;
  p->x += dm;
}

int coarse_shift_diag(long Vc, int n, double2 *Y, double dm, hipStream_t st) {
  hipLaunchKernelGGL(k_shift_diag, dim3((unsigned)((Vc * n + TB - 1) / TB)), dim3(TB), 0, st, Vc, n, Y, dm);
  WMG_HIP(hipGetLastError());
  return 0;
}

__global__ void k_Y_to_float(size_t cnt, const double2 *Y, float2 *Yf) {
  size_t i = blockIdx.x * (size_t)TB + threadIdx.x;
  if (i < cnt) Yf[i] = make_float2((float)Y[i].x, (float)Y[i].y);
}

int coarse_convert(long count, const double2 *Y64, int yprec, void *Yout, hipStream_t st) {
  if (yprec != P32) return set_error(-1, "coarse_convert: precision %d", yprec);
  hipLaunchKernelGGL(k_Y_to_float, dim3((unsigned)((count + TB - 1) / TB)), dim3(TB), 0, st, (size_t)count, Y64,
                     (float2 *)Yout);
  WMG_HIP(hipGetLastError());
  return 0;
}

// internal [xh][d][col][row] <-> canonical [xh][d][row][col]
__global__ void k_Y_transpose(long nblk, int n, const double2 *a, double2 *b) {
  size_t i = blockIdx.x * (size_t)TB + threadIdx.x;
  size_t tot = (size_t)nblk * n * n;
  if (i >= tot) return;
  size_t blk = i / ((size_t)n * n);
  int rr = (int)((i / n) % n), cc = (int)(i % n);
  b[blk * n * n + (size_t)cc * n + rr] = a[i];
}

int coarse_transpose(long nblk, int n, const double2 *a, double2 *b, hipStream_t st) {
  size_t tot = (size_t)nblk * n * n;
  hipLaunchKernelGGL(k_Y_transpose, dim3((unsigned)((tot + TB - 1) / TB)), dim3(TB), 0, st, nblk, n, a, b);
  WMG_HIP(hipGetLastError());
  return 0;
}


// ------------------------------------------------------------ MFMA apply
// Multi-RHS coarse stencil on the matrix cores.  Per coarse site and
// direction the complex block product C = Y B (Y: n x n link block, B: the
// neighbour's n x R vectors of R right-hand sides) is written as one real
// GEMM without duplicating the links:
//   [Cr | Ci] (n x 2R) = [Yr | Yi] (n x 2n) . [[Br, Bi], [-Bi, Br]] (2n x 2R)
// and accumulated over the nine directions with v_mfma_f32_16x16x4f32.  One
// workgroup per site, one wavefront per 16-row tile of the output.  The A
// operand streams from a pre-swizzled FP32 copy of the links laid out
// [site][d][row tile][k-step/4][lane][k-step%4] with the k-steps padded to a
// multiple of 8 by zeros (each lane reads four k-steps with one 16-byte
// load, a wavefront 1 KB contiguous; every link byte is read once); the B operand of each
// direction is staged in LDS.  Lane layout of the 16x16x4 instruction: lane
// l supplies A[l%16][l/16] and B[l/16][l%16]; accumulator register v of lane
// l holds C[4*(l/16)+v][l%16].
typedef float floatx4 __attribute__((ext_vector_type(4)));

// k-steps of the MFMA link layout for n x n blocks: n/2 rounded up to 8
__host__ __device__ __forceinline__ int mfma_km(int n) { return (n / 2 + 7) / 8 * 8; }

__global__ void k_Y_to_mfma(long Vc, int n, int MT, int KM, const double2 *__restrict__ Y, float *__restrict__ Ym) {
  size_t i = blockIdx.x * (size_t)TB + threadIdx.x;
  size_t per_site_d = (size_t)MT * KM * 64;
  size_t tot = (size_t)Vc * 9 * per_site_d;
  if (i >= tot) return;
  size_t sd = i / per_site_d;  // site*9 + d
  size_t rem = i % per_site_d;
  int mt = (int)(rem / ((size_t)KM * 64));
  int q = (int)(rem % ((size_t)KM * 64));  // (kq*64 + lane)*4 + e
  int e = q % 4, lane = (q / 4) % 64, kq = q / 256;
  int ks = kq * 4 + e;
  int row = mt * 16 + lane % 16, kk = ks * 4 + lane / 16;
  float v = 0.f;
  if (row < n && kk < 2 * n) {
    int col = kk < n ? kk : kk - n;
    double2 y = Y[(sd * n + col) * n + row];  // internal [site][d][col][row]
    v = (float)(kk < n ? y.x : y.y);
  }
  Ym[i] = v;
}

int coarse_to_mfma(long Vc, int n, const double2 *Y64, float *Ym, hipStream_t st) {
  int MT = (n + 15) / 16, KM = mfma_km(n);
  size_t tot = (size_t)Vc * 9 * MT * KM * 64;
  hipLaunchKernelGGL(k_Y_to_mfma, dim3((unsigned)((tot + TB - 1) / TB)), dim3(TB), 0, st, Vc, n, MT, KM, Y64, Ym);
  WMG_HIP(hipGetLastError());
  return 0;
}

size_t coarse_mfma_floats(long Vc, int n) { return (size_t)Vc * 9 * ((n + 15) / 16) * mfma_km(n) * 64; }

size_t coarse_mfma_halfs(long Vc, int n) { return coarse_mfma_floats(Vc, n); }

// FP16 copy of the swizzled links: one workgroup per (site, direction)
// block; its scale is the largest |re| or |im| of the block (1 for a zero
// block), entries are stored as RNE(y / scale)
__global__ void __launch_bounds__(TB) k_Y_to_mfma16(int n, int MT, int KM, const double2 *__restrict__ Y,
                                                   __half *__restrict__ Yh, float *__restrict__ Ysc) {
  const size_t sd = blockIdx.x;  // site*9 + d
  const double2 *blk = Y + sd * (size_t)n * n;
  double mx = 0;
  for (int i = threadIdx.x; i < n * n; i += TB) mx = fmax(mx, fmax(fabs(blk[i].x), fabs(blk[i].y)));
  __shared__ double sh[TB / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_down(mx, o, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = mx;
  __syncthreads();
  double scale = sh[0];
  for (int w = 1; w < TB / 64; w++) scale = fmax(scale, sh[w]);
  if (!(scale > 0)) scale = 1.0;
  const double inv = 1.0 / scale;
  if (threadIdx.x == 0) Ysc[sd] = (float)scale;
  const size_t per = (size_t)MT * KM * 64;
  for (size_t rem = threadIdx.x; rem < per; rem += TB) {
    int mt = (int)(rem / ((size_t)KM * 64));
    int q = (int)(rem % ((size_t)KM * 64));
    int e = q % 4, lane = (q / 4) % 64, kq = q / 256;
    int ks = kq * 4 + e;
    int row = mt * 16 + lane % 16, kk = ks * 4 + lane / 16;
    float v = 0.f;
    if (row < n && kk < 2 * n) {
      int col = kk < n ? kk : kk - n;
      double2 y = blk[(size_t)col * n + row];  // internal [site][d][col][row]
      v = (float)((kk < n ? y.x : y.y) * inv);
    }
    Yh[sd * per + rem] = __float2half_rn(v);
  }
}

int coarse_to_mfma16(long Vc, int n, const double2 *Y64, __half *Yh, float *Ysc, hipStream_t st) {
  int MT = (n + 15) / 16, KM = mfma_km(n);
  hipLaunchKernelGGL(k_Y_to_mfma16, dim3((unsigned)(Vc * 9)), dim3(TB), 0, st, n, MT, KM, Y64, Yh, Ysc);
  WMG_HIP(hipGetLastError());
  return 0;
}

// LDS row stride of the transposed B tile: a multiple of 32 plus 4, so the
// 16 columns x 4 k-rows read by one MFMA B fragment spread over all banks
__host__ __device__ __forceinline__ int mfma_ldk(int n) { return (2 * n + 31) / 32 * 32 + 4; }
// ... of the k-step-contiguous tile of k_coarse_apply_mfma2 (n a multiple of
// 8): 2n + 4 floats, four times an odd number modulo 64, so the 16 columns
// of a 16-lane group of 16-byte reads start in distinct bank quadruples
__host__ __device__ __forceinline__ int mfma2_ldk(int n) { return 2 * n + 4; }

// One workgroup per (coarse site, tile of up to 32 right-hand sides); wave mt
// owns rows 16mt..16mt+15 of the n x n blocks and all NT column tiles.  The
// loop over the 9 stencil directions is software pipelined: while the MFMAs
// of direction d run, the link fragments of direction d+1 (registers) and
// its neighbour vectors (registers, written to LDS after the next barrier)
// are already in flight, so no direction waits for a cold load.
template <int NT, int KM, bool AH>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
k_coarse_apply_mfma(const float *__restrict__ Ym, const __half *__restrict__ Yh, const float *__restrict__ Ysc,
                    const float2 *__restrict__ in, float2 *__restrict__ out, int L0, int L1, int L2, int L3, long Vc,
                    int n, int nrhs, int dagger) {
  extern __shared__ float Bt[];  // B transposed: [NT*16 columns][LDK], column j, k-row kk at j*LDK + kk
  const int LDK = mfma_ldk(n);
  const int MT = (n + 15) / 16;
  long xh = blockIdx.x;
  int r0 = blockIdx.y * 32;
  int R = nrhs - r0 < 32 ? nrhs - r0 : 32;
  int mt = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int L[4] = {L0, L1, L2, L3};
  int x[4];
  site_coords(L, xh, x);
  // neighbour site of direction d (0: the site, 1+mu: +mu, 5+mu: -mu)
  auto nbr = [&](int d) -> long {
    if (d == 0) return xh;
    int mu = (d - 1) & 3;
    int y[4] = {x[0], x[1], x[2], x[3]};
    y[mu] = d < 5 ? (x[mu] + 1) % L[mu] : (x[mu] - 1 + L[mu]) % L[mu];
    return site_index(L, y);
  };
  const int h = n / 2, NC = NT * 16;
  // padding columns 2R..NC-1 and padding k-rows 2n..4KM-1 stay zero for
  // every direction (4KM <= LDK - 4)
  for (int idx = threadIdx.x; idx < (NC - 2 * R) * LDK; idx += blockDim.x) Bt[2 * R * LDK + idx] = 0.f;
  for (int idx = threadIdx.x; idx < 2 * R * (4 * KM - 2 * n); idx += blockDim.x) {
    int j = idx / (4 * KM - 2 * n), kk = 2 * n + idx % (4 * KM - 2 * n);
    Bt[j * LDK + kk] = 0.f;
  }
  // staging map: thread -> (column col, rows rg, rg + tpr, ...); tpr >= 4
  // row groups fit in 64*MT threads, so 8 rounds cover R <= 32 rows
  const int tpr = (int)blockDim.x / n;
  const int col = threadIdx.x % n, rg = threadIdx.x / n;
  const bool stager = rg < tpr;
  const bool neg = dagger && col >= h;
  float2 stg[8];
  auto stage_load = [&](int d) {
    const float2 *src = in + ((size_t)(r0 + rg) * Vc + nbr(d)) * n + col;
    const size_t step = (size_t)tpr * Vc * n;
#pragma unroll
    for (int q = 0; q < 8; q++)
      if (stager && rg + q * tpr < R) stg[q] = src[q * step];
  };
  // B = [[Br, Bi], [-Bi, Br]] (col fastest across threads: conflict-free writes)
  auto stage_store = [&]() {
    float *dst = Bt + rg * LDK + col;
#pragma unroll
    for (int q = 0; q < 8; q++)
      if (stager && rg + q * tpr < R) {
        float2 v = stg[q];
        if (neg) { v.x = -v.x; v.y = -v.y; }
        float *p = dst + q * tpr * LDK;
        p[0] = v.x;
        p[R * LDK] = v.y;
        p[n] = -v.y;
        p[R * LDK + n] = v.x;
      }
  };
  const int mts = mt < MT ? mt : 0;
  auto a_load = [&](float *a, int d) {
    if constexpr (AH) {
      // four k-steps as four halves (8 bytes) per lane, scaled back
      const float sc = Ysc[(size_t)xh * 9 + d];
      const uint2 *Ad = (const uint2 *)(Yh + (((size_t)xh * 9 + d) * MT + mts) * KM * 64) + lane;
#pragma unroll
      for (int kq = 0; kq < KM / 4; kq++) {
        uint2 v = Ad[kq * 64];
        float2 f01 = __half22float2(*(const __half2 *)&v.x), f23 = __half22float2(*(const __half2 *)&v.y);
        a[4 * kq] = f01.x * sc;
        a[4 * kq + 1] = f01.y * sc;
        a[4 * kq + 2] = f23.x * sc;
        a[4 * kq + 3] = f23.y * sc;
      }
    } else {
      const float4 *Ad = (const float4 *)(Ym + (((size_t)xh * 9 + d) * MT + mts) * KM * 64) + lane;
#pragma unroll
      for (int kq = 0; kq < KM / 4; kq++) {
        float4 v = Ad[kq * 64];
        a[4 * kq] = v.x;
        a[4 * kq + 1] = v.y;
        a[4 * kq + 2] = v.z;
        a[4 * kq + 3] = v.w;
      }
    }
  };
  floatx4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; t++) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  float a_cur[KM], a_nxt[KM];
  stage_load(0);
  a_load(a_cur, 0);
  for (int d = 0; d < 9; d++) {
    __syncthreads();  // every wave is done reading B of direction d-1
    stage_store();
    __syncthreads();
    if (d + 1 < 9) {
      stage_load(d + 1);
      a_load(a_nxt, d + 1);
    }
    if (mt < MT) {
      const int krow = lane >> 4, jc = lane & 15;
#pragma unroll
      for (int ks = 0; ks < KM; ks++) {
        // k-steps KS..KM-1 multiply zero link fragments with zero B rows:
        // a fixed trip count keeps the accumulators in place
        const float *bcol = Bt + jc * LDK + ks * 4 + krow;
#pragma unroll
        for (int t = 0; t < NT; t++)
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_cur[ks], bcol[t * 16 * LDK], acc[t], 0, 0, 0);
      }
    }
#pragma unroll
    for (int ks = 0; ks < KM; ks++) a_cur[ks] = a_nxt[ks];
  }
  if (mt >= MT) return;
  float *of = (float *)out;
#pragma unroll
  for (int t = 0; t < NT; t++)
#pragma unroll
    for (int v = 0; v < 4; v++) {
      int row = mt * 16 + 4 * (lane >> 4) + v, j = t * 16 + (lane & 15);
      if (row < n && j < 2 * R) {
        int r = j < R ? j : j - R;
        float val = acc[t][v];
        if (dagger && row >= h) val = -val;
        of[2 * (((size_t)(r0 + r) * Vc + xh) * n + row) + (j < R ? 0 : 1)] = val;
      }
    }
}

// Variant for n = N in {32, 40, 48, 64} that stages each neighbour value
// once: with B = [Br; Bi] (2n x R, no duplication) the real and imaginary
// parts of C are two GEMMs over the same B,
//   Cr = [Yr | -Yi] B,   Ci = [Yi | Yr] B,
// and both A operands are the stored fragments [Yr | Yi] of the wave's
// registers: for k-step ks (4 k each, Q = N/4 k-steps per half) the first
// is S(ks) or -S(ks), the second S(ks + Q) or S(ks - Q).  Half the LDS
// writes and reads of the duplicated form, the same MFMA count, and C
// comes out as (re, im) pairs per lane.
template <int NTR, int N, bool AH>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5)))
k_coarse_apply_mfma2(const float *__restrict__ Ym, const __half *__restrict__ Yh, const float *__restrict__ Ysc,
                     const float2 *__restrict__ in, float2 *__restrict__ out, int L0, int L1, int L2, int L3, long Vc,
                     int nrhs, int dagger, double *__restrict__ npart) {
  constexpr int KM = (N / 2 + 7) / 8 * 8;  // k-steps of the stored fragments
  constexpr int KS = N / 2, Q = N / 4;     // k-steps used; per half
  constexpr int MT = (N + 15) / 16;
  extern __shared__ float Bt[];  // [NTR*16 columns][LDK]; see stage_store for the k order
  const int LDK = mfma2_ldk(N);
  long xh = blockIdx.x;
  int r0 = blockIdx.y * 32;
  int R = nrhs - r0 < 32 ? nrhs - r0 : 32;
  int mt = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int L[4] = {L0, L1, L2, L3};
  int x[4];
  site_coords(L, xh, x);
  auto nbr = [&](int d) -> long {
    if (d == 0) return xh;
    int mu = (d - 1) & 3;
    int y[4] = {x[0], x[1], x[2], x[3]};
    y[mu] = d < 5 ? (x[mu] + 1) % L[mu] : (x[mu] - 1 + L[mu]) % L[mu];
    return site_index(L, y);
  };
  constexpr int h = N / 2;
  // padding columns R..16 NTR - 1 stay zero for every direction
  for (int idx = threadIdx.x; idx < (NTR * 16 - R) * LDK; idx += blockDim.x) Bt[R * LDK + idx] = 0.f;
  constexpr int tpr = 64 * MT / N;  // >= 4 row groups: 8 rounds cover R <= 32
  const int col = threadIdx.x % N, rg = threadIdx.x / N;
  const bool stager = rg < tpr;
  const bool neg = dagger && col >= h;
  float2 stg[8];
  auto stage_load = [&](int d) {
    const float2 *src = in + ((size_t)(r0 + rg) * Vc + nbr(d)) * N + col;
    const size_t step = (size_t)tpr * Vc * N;
#pragma unroll
    for (int q = 0; q < 8; q++)
      if (stager && rg + q * tpr < R) stg[q] = src[q * step];
  };
  // B row k of column r lives at r*LDK + (k % 4)*KS + k/4: the KS k-steps a
  // lane multiplies (k = 4 ks + krow) are contiguous, four per 16-byte read
  auto stage_store = [&]() {
    float *dst = Bt + rg * LDK + (col % 4) * KS + col / 4;
#pragma unroll
    for (int q = 0; q < 8; q++)
      if (stager && rg + q * tpr < R) {
        float2 v = stg[q];
        if (neg) { v.x = -v.x; v.y = -v.y; }
        dst[q * tpr * LDK] = v.x;           // k = col
        dst[q * tpr * LDK + N / 4] = v.y;   // k = N + col (N % 4 == 0)
      }
  };
  const int mts = mt < MT ? mt : 0;
  auto a_load = [&](float *a, int d) {
    if constexpr (AH) {
      const float sc = Ysc[(size_t)xh * 9 + d];
      const uint2 *Ad = (const uint2 *)(Yh + (((size_t)xh * 9 + d) * MT + mts) * KM * 64) + lane;
#pragma unroll
      for (int kq = 0; kq < KS / 4; kq++) {
        uint2 v = Ad[kq * 64];
        float2 f01 = __half22float2(*(const __half2 *)&v.x), f23 = __half22float2(*(const __half2 *)&v.y);
        a[4 * kq] = f01.x * sc;
        a[4 * kq + 1] = f01.y * sc;
        a[4 * kq + 2] = f23.x * sc;
        a[4 * kq + 3] = f23.y * sc;
      }
    } else {
      const float4 *Ad = (const float4 *)(Ym + (((size_t)xh * 9 + d) * MT + mts) * KM * 64) + lane;
#pragma unroll
      for (int kq = 0; kq < KS / 4; kq++) {
        float4 v = Ad[kq * 64];
        a[4 * kq] = v.x;
        a[4 * kq + 1] = v.y;
        a[4 * kq + 2] = v.z;
        a[4 * kq + 3] = v.w;
      }
    }
  };
  floatx4 cr[NTR], ci[NTR];
#pragma unroll
  for (int t = 0; t < NTR; t++) cr[t] = ci[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  float a_cur[KS], a_nxt[KS];
  stage_load(0);
  a_load(a_cur, 0);
  const int krow = lane >> 4, jc = lane & 15;
  for (int d = 0; d < 9; d++) {
    __syncthreads();  // every wave is done reading B of direction d-1
    stage_store();
    __syncthreads();
    if (d + 1 < 9) {
      stage_load(d + 1);
      a_load(a_nxt, d + 1);
    }
    if (mt < MT) {
      const float *bcol = Bt + jc * LDK + krow * KS;
#pragma unroll
      for (int k4 = 0; k4 < KS; k4 += 4) {
        float4 bv[NTR];
#pragma unroll
        for (int t = 0; t < NTR; t++) bv[t] = *(const float4 *)(bcol + t * 16 * LDK + k4);
#pragma unroll
        for (int u = 0; u < 4; u++) {
          const int ks = k4 + u;
          const float a1 = ks < Q ? a_cur[ks] : -a_cur[ks];
          const float a2 = ks < Q ? a_cur[ks + Q] : a_cur[ks - Q];
#pragma unroll
          for (int t = 0; t < NTR; t++) {
            const float b = u == 0 ? bv[t].x : (u == 1 ? bv[t].y : (u == 2 ? bv[t].z : bv[t].w));
            cr[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b, cr[t], 0, 0, 0);
            ci[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a2, b, ci[t], 0, 0, 0);
          }
        }
      }
    }
#pragma unroll
    for (int ks = 0; ks < KS; ks++) a_cur[ks] = a_nxt[ks];
  }
  // the block has exactly MT waves: every wave reaches the barrier below
#pragma unroll
  for (int t = 0; t < NTR; t++)
#pragma unroll
    for (int v = 0; v < 4; v++) {
      const int row = mt * 16 + 4 * (lane >> 4) + v, r = t * 16 + (lane & 15);
      if (row < N && r < R) {
        float2 val = make_float2(cr[t][v], ci[t][v]);
        if (dagger && row >= h) { val.x = -val.x; val.y = -val.y; }
        out[((size_t)(r0 + r) * Vc + xh) * N + row] = val;
      }
    }
  if (npart) {
    // |out|^2 of this site per rhs: the wave's rows, then the MT waves in order
    __shared__ double nsh[MT][NTR * 16];
#pragma unroll
    for (int t = 0; t < NTR; t++) {
      double q = 0;
#pragma unroll
      for (int v = 0; v < 4; v++) {
        const int row = mt * 16 + 4 * (lane >> 4) + v;
        if (row < N) q += (double)cr[t][v] * cr[t][v] + (double)ci[t][v] * ci[t][v];
      }
      q += __shfl_xor(q, 16, 64);
      q += __shfl_xor(q, 32, 64);
      if (lane < 16) nsh[mt][t * 16 + lane] = q;
    }
    __syncthreads();
    if ((int)threadIdx.x < R) {
      double q = 0;
#pragma unroll
      for (int m = 0; m < MT; m++) q += nsh[m][threadIdx.x];
      npart[(size_t)(r0 + threadIdx.x) * Vc + xh] = q;
    }
  }
}

// ---- FP16 products
// With FP16 links the stencil can also multiply in FP16
// (v_mfma_f32_16x16x16f16: one instruction takes the four k-steps a lane
// holds, 4x fewer matrix instructions than FP32 products), accumulating in
// FP32.  B = the neighbour vector times the block's link scale, rounded to
// FP16, with one power-of-two scale per right-hand side that brings its
// largest |re| or |im| to [1024, 2048): the products keep FP16's 11 bits
// relative to each rhs's largest entry (the stored links already round at
// 2^-11 of their block's largest entry) and cannot overflow (link entries
// scaled to |y| <= 1, block scales of order 1).

// partial maxima of |re|, |im| of each rhs's vector: EMX per rhs
constexpr int EMX = COARSE_H_PART;
__global__ void __launch_bounds__(256) k_rhs_absmax(const float2 *__restrict__ v, long len, float *__restrict__ part) {
  const int r = blockIdx.y, j = blockIdx.x;
  const float2 *p = v + (size_t)r * len;
  float m = 0.f;
  for (long i = (long)j * 256 + threadIdx.x; i < len; i += (long)EMX * 256) {
    const float2 x = p[i];
    m = fmaxf(m, fmaxf(fabsf(x.x), fabsf(x.y)));
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_down(m, o, 64));
  __shared__ float sh[4];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) part[(size_t)r * EMX + j] = fmaxf(fmaxf(sh[0], sh[1]), fmaxf(sh[2], sh[3]));
}

int rhs_absmax(const float2 *v, long len, int nrhs, float *part, hipStream_t st) {
  hipLaunchKernelGGL(k_rhs_absmax, dim3(EMX, nrhs), dim3(256), 0, st, v, len, part);
  WMG_HIP(hipGetLastError());
  return 0;
}

typedef _Float16 half4 __attribute__((ext_vector_type(4)));
// k_coarse_apply_mfma2 with FP16 products (same tiling, fragments, B order
// and epilogue): the lane's four consecutive k-steps of A (as stored) and of
// B (one 8-byte LDS read) are one FP16 fragment; the k order inside the
// instruction is permuted the same way for both operands.
template <int NTR, int N>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5)))
k_coarse_apply_mfma2h(const __half *__restrict__ Yh, const float *__restrict__ Ysc, const float2 *__restrict__ in,
                      float2 *__restrict__ out, int L0, int L1, int L2, int L3, long Vc, int nrhs, int dagger,
                      double *__restrict__ npart, const float *__restrict__ bpart) {
  constexpr int KM = (N / 2 + 7) / 8 * 8;
  constexpr int KS = N / 2, Q = N / 4;
  constexpr int MT = (N + 15) / 16;
  constexpr int LDKH = 2 * N + 8;  // halves per B column
  static_assert(Q % 4 == 0, "the sign switch of [Yr | -Yi] must fall between fragments");
  extern __shared__ _Float16 Bh[];  // [NTR*16 columns][LDKH], k order of k_coarse_apply_mfma2
  __shared__ float bsh[32];         // per-rhs scale
  long xh = blockIdx.x;
  int r0 = blockIdx.y * 32;
  int R = nrhs - r0 < 32 ? nrhs - r0 : 32;
  int mt = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int L[4] = {L0, L1, L2, L3};
  int x[4];
  site_coords(L, xh, x);
  auto nbr = [&](int d) -> long {
    if (d == 0) return xh;
    int mu = (d - 1) & 3;
    int y[4] = {x[0], x[1], x[2], x[3]};
    y[mu] = d < 5 ? (x[mu] + 1) % L[mu] : (x[mu] - 1 + L[mu]) % L[mu];
    return site_index(L, y);
  };
  constexpr int h = N / 2;
  if ((int)threadIdx.x < R) {
    float m = 0.f;
    for (int j = 0; j < EMX; j++) m = fmaxf(m, bpart[(size_t)(r0 + threadIdx.x) * EMX + j]);
    int e = 0;
    (void)frexpf(m, &e);
    const int k = 11 - e < -126 ? -126 : (11 - e > 126 ? 126 : 11 - e);
    bsh[threadIdx.x] = m > 0.f ? ldexpf(1.f, k) : 1.f;
  }
  for (int idx = threadIdx.x; idx < (NTR * 16 - R) * LDKH; idx += blockDim.x) Bh[R * LDKH + idx] = (_Float16)0.f;
  constexpr int tpr = 64 * MT / N;
  const int col = threadIdx.x % N, rg = threadIdx.x / N;
  const bool stager = rg < tpr;
  const bool neg = dagger && col >= h;
  float2 stg[8];
  auto stage_load = [&](int d) {
    const float2 *src = in + ((size_t)(r0 + rg) * Vc + nbr(d)) * N + col;
    const size_t step = (size_t)tpr * Vc * N;
#pragma unroll
    for (int q = 0; q < 8; q++)
      if (stager && rg + q * tpr < R) stg[q] = src[q * step];
  };
  // B row k of column r at r*LDKH + (k % 4)*KS + k/4, times the link block
  // scale and the rhs scale, in FP16
  auto stage_store = [&](float sc) {
    _Float16 *dst = Bh + rg * LDKH + (col % 4) * KS + col / 4;
#pragma unroll
    for (int q = 0; q < 8; q++)
      if (stager && rg + q * tpr < R) {
        const float2 v = stg[q];
        const float s = (neg ? -sc : sc) * bsh[rg + q * tpr];
        dst[q * tpr * LDKH] = (_Float16)(v.x * s);
        dst[q * tpr * LDKH + N / 4] = (_Float16)(v.y * s);
      }
  };
  const int mts = mt < MT ? mt : 0;
  // the links stream through once per launch: non-temporal loads leave L2
  // to the neighbour vectors, which nine workgroups read
  auto a_load = [&](half4 *a, int d) {
    typedef unsigned u32x2_t __attribute__((ext_vector_type(2)));
    const u32x2_t *Ad = (const u32x2_t *)(Yh + (((size_t)xh * 9 + d) * MT + mts) * KM * 64) + lane;
#pragma unroll
    for (int kq = 0; kq < KS / 4; kq++) {
      const u32x2_t v = __builtin_nontemporal_load(Ad + kq * 64);
      __builtin_memcpy(&a[kq], &v, 8);
    }
  };
  floatx4 cr[NTR], ci[NTR];
#pragma unroll
  for (int t = 0; t < NTR; t++) cr[t] = ci[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  half4 a_cur[KS / 4], a_nxt[KS / 4];
  float sc_cur = Ysc[(size_t)xh * 9], sc_nxt = 0.f;
  stage_load(0);
  a_load(a_cur, 0);
  const int krow = lane >> 4, jc = lane & 15;
  for (int d = 0; d < 9; d++) {
    __syncthreads();  // every wave is done reading B of direction d-1 (and bsh is written)
    stage_store(sc_cur);
    __syncthreads();
    if (d + 1 < 9) {
      stage_load(d + 1);
      a_load(a_nxt, d + 1);
      sc_nxt = Ysc[(size_t)xh * 9 + d + 1];
    }
    if (mt < MT) {
      const _Float16 *bcol = Bh + jc * LDKH + krow * KS;
#pragma unroll
      for (int b = 0; b < KS / 4; b++) {
        // [Yr | -Yi] and [Yi | Yr] from the stored [Yr | Yi]
        const half4 a1 = b < Q / 4 ? a_cur[b] : -a_cur[b];
        const half4 a2 = b < Q / 4 ? a_cur[b + Q / 4] : a_cur[b - Q / 4];
#pragma unroll
        for (int t = 0; t < NTR; t++) {
          half4 bv;
          __builtin_memcpy(&bv, bcol + t * 16 * LDKH + 4 * b, 8);
          cr[t] = __builtin_amdgcn_mfma_f32_16x16x16f16(a1, bv, cr[t], 0, 0, 0);
          ci[t] = __builtin_amdgcn_mfma_f32_16x16x16f16(a2, bv, ci[t], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int kq = 0; kq < KS / 4; kq++) a_cur[kq] = a_nxt[kq];
    sc_cur = sc_nxt;
  }
#pragma unroll
  for (int t = 0; t < NTR; t++) {
    const int r = t * 16 + (lane & 15);
    const float inv = r < R ? 1.f / bsh[r] : 0.f;
#pragma unroll
    for (int v = 0; v < 4; v++) {
      cr[t][v] *= inv;
      ci[t][v] *= inv;
      const int row = mt * 16 + 4 * (lane >> 4) + v;
      if (row < N && r < R) {
        float2 val = make_float2(cr[t][v], ci[t][v]);
        if (dagger && row >= h) { val.x = -val.x; val.y = -val.y; }
        out[((size_t)(r0 + r) * Vc + xh) * N + row] = val;
      }
    }
  }
  if (npart) {
    __shared__ double nsh[MT][NTR * 16];
#pragma unroll
    for (int t = 0; t < NTR; t++) {
      double q = 0;
#pragma unroll
      for (int v = 0; v < 4; v++) {
        const int row = mt * 16 + 4 * (lane >> 4) + v;
        if (row < N) q += (double)cr[t][v] * cr[t][v] + (double)ci[t][v] * ci[t][v];
      }
      q += __shfl_xor(q, 16, 64);
      q += __shfl_xor(q, 32, 64);
      if (lane < 16) nsh[mt][t * 16 + lane] = q;
    }
    __syncthreads();
    if ((int)threadIdx.x < R) {
      double q = 0;
#pragma unroll
      for (int m = 0; m < MT; m++) q += nsh[m][threadIdx.x];
      npart[(size_t)(r0 + threadIdx.x) * Vc + xh] = q;
    }
  }
}

static int coarse_apply_mfma_any(const Geom &gc, int n, const float *Ym, const __half *Yh, const float *Ysc,
                                 const float2 *in, float2 *out, int dagger, int nrhs, hipStream_t st,
                                 double *npart = nullptr, bool *fused = nullptr, float *bpart = nullptr) {
  if (fused) *fused = false;
  if (n > 64 || (n & 1)) return set_error(-1, "coarse_apply_mfma: n=%d (even, <= 64)", n);
  int MT = (n + 15) / 16;
  int rmax = nrhs < 32 ? nrhs : 32;
  int NT = (2 * rmax + 15) / 16;
  dim3 grid((unsigned)gc.V, (nrhs + 31) / 32);
  dim3 blk(64 * MT);
  // (n / 4 a multiple of 4: the sign switch of [Yr | -Yi] falls between
  // the four-k-step fragments)
  if (Yh && bpart && (n == 32 || n == 48 || n == 64)) {
    const int NTR = (rmax + 15) / 16;
    const size_t ldsh = sizeof(_Float16) * NTR * 16 * (2 * n + 8);
    hipLaunchKernelGGL(k_rhs_absmax, dim3(EMX, nrhs), dim3(256), 0, st, in, gc.V * n, bpart);
#define H_CASE(T, NN)                                                                                        \
  if (NTR == T && n == NN) {                                                                                \
    hipLaunchKernelGGL((k_coarse_apply_mfma2h<T, NN>), grid, blk, ldsh, st, Yh, Ysc, in, out, gc.L[0], gc.L[1], \
                       gc.L[2], gc.L[3], gc.V, nrhs, dagger, npart, (const float *)bpart);                  \
    WMG_HIP(hipGetLastError());                                                                             \
    if (fused) *fused = npart != nullptr;                                                                   \
    return 0;                                                                                               \
  }
    H_CASE(1, 32) H_CASE(1, 48) H_CASE(1, 64)
    H_CASE(2, 32) H_CASE(2, 48) H_CASE(2, 64)
#undef H_CASE
  }
  if (n == 32 || n == 40 || n == 48 || n == 64) {
    const int NTR = (rmax + 15) / 16;
    size_t lds2 = sizeof(float) * NTR * 16 * mfma2_ldk(n);
#define N2_CASE(T, NN)                                                                                         \
  if (NTR == T && n == NN) {                                                                                  \
    if (Yh)                                                                                                   \
      hipLaunchKernelGGL((k_coarse_apply_mfma2<T, NN, true>), grid, blk, lds2, st, Ym, Yh, Ysc, in, out,       \
                         gc.L[0], gc.L[1], gc.L[2], gc.L[3], gc.V, nrhs, dagger, npart);                      \
    else                                                                                                      \
      hipLaunchKernelGGL((k_coarse_apply_mfma2<T, NN, false>), grid, blk, lds2, st, Ym, Yh, Ysc, in, out,      \
                         gc.L[0], gc.L[1], gc.L[2], gc.L[3], gc.V, nrhs, dagger, npart);                      \
    WMG_HIP(hipGetLastError());                                                                               \
    if (fused) *fused = npart != nullptr;                                                                     \
    return 0;                                                                                                 \
  }
    N2_CASE(1, 32) N2_CASE(1, 40) N2_CASE(1, 48) N2_CASE(1, 64)
    N2_CASE(2, 32) N2_CASE(2, 40) N2_CASE(2, 48) N2_CASE(2, 64)
#undef N2_CASE
  }
  size_t lds = sizeof(float) * NT * 16 * mfma_ldk(n);
  const int KM = mfma_km(n);  // 8, 16, 24 or 32
#define NT_CASE(N, K)                                                                                           \
  if (NT == N && KM == K) {                                                                                    \
    if (Yh)                                                                                                    \
      hipLaunchKernelGGL((k_coarse_apply_mfma<N, K, true>), grid, blk, lds, st, Ym, Yh, Ysc, in, out, gc.L[0],  \
                         gc.L[1], gc.L[2], gc.L[3], gc.V, n, nrhs, dagger);                                   \
    else                                                                                                       \
      hipLaunchKernelGGL((k_coarse_apply_mfma<N, K, false>), grid, blk, lds, st, Ym, Yh, Ysc, in, out, gc.L[0], \
                         gc.L[1], gc.L[2], gc.L[3], gc.V, n, nrhs, dagger);                                   \
  } else
#define NT_ALL(N) NT_CASE(N, 8) NT_CASE(N, 16) NT_CASE(N, 24) NT_CASE(N, 32)
  NT_ALL(1) NT_ALL(2) NT_ALL(3) NT_ALL(4)
  return set_error(-1, "coarse_apply_mfma: NT=%d KM=%d", NT, KM);
#undef NT_ALL
#undef NT_CASE
  WMG_HIP(hipGetLastError());
  return 0;
}

int coarse_apply_mfma(const Geom &gc, int n, const float *Ym, const float2 *in, float2 *out, int dagger, int nrhs,
                      hipStream_t st, double *npart, bool *fused) {
  return coarse_apply_mfma_any(gc, n, Ym, nullptr, nullptr, in, out, dagger, nrhs, st, npart, fused);
}

int coarse_apply_mfma16(const Geom &gc, int n, const __half *Yh, const float *Ysc, const float2 *in, float2 *out,
                        int dagger, int nrhs, hipStream_t st, double *npart, bool *fused, float *bpart) {
  if (!Yh || !Ysc) return set_error(-1, "coarse_apply_mfma16: null links");
  if (bpart && nrhs > COARSE_H_MAXRHS) return set_error(-1, "coarse_apply_mfma16: FP16 products for at most %d rhs",
                                                        COARSE_H_MAXRHS);
  return coarse_apply_mfma_any(gc, n, nullptr, Yh, Ysc, in, out, dagger, nrhs, st, npart, fused, bpart);
}

}  // namespace wmg
