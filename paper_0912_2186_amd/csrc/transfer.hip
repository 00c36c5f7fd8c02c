// Inter-grid transfer of the adaptive multigrid (arXiv:0912.2186, Sec. 2-3):
//   * random start vectors of the adaptive setup (Philox4x32-10)
//   * block orthonormalisation of the null vectors, Eq. 2.7, split by
//     chirality so that sigma_3 P = P gamma_5 (Sec. 3)
//   * restriction r_hat = P^dag r and prolongation e = P e_hat (Eq. 2.3)
//
// The prolongator is stored block-major, [alpha][xh][block element], so one
// workgroup reads the whole aggregate of a coarse site as a contiguous slab.
// A block element e enumerates (fine site k of the block, component c):
//   fine lattice (SoA spinors):   e = c * bs + k   (sites fastest)
//   coarse lattice (AoS vectors): e = k * dof + c  (components fastest)
// Chirality of component c is c / (dof/2).  In FP16 storage every
// (alpha, xh, k) site of P carries one FP32 scale (max |re|, |im| of its
// components), the stored halves being the components divided by it.
#include <cstdio>

#include "wmg_internal.h"

namespace wmg {

static constexpr int TB = 256;

// ------------------------------------------------------------ Philox4x32-10
// Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3"
// (SC'11): 10 rounds of two 32x32->64 multiplies with the Weyl key schedule.
__device__ __forceinline__ void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; r++) {
    uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
    uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
    uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// Vector alpha of level lvl: component (s, c) = (int32(w0), int32(w1)) * 2^-31
// with w = Philox(ctr = (c, s, alpha, lvl), key = seed).  Written in the
// level's vector layout (fine: SoA [12][V]; coarse: AoS [V][dof]).
__global__ void k_start_vectors(long nsite, int dof, uint32_t k0, uint32_t k1, int lvl, int alpha0, double2 *out,
                                int fine_soa, long Vs) {
  long i = blockIdx.x * (long)TB + threadIdx.x;
  int a = blockIdx.y;
  if (i >= nsite * dof) return;
  long s, c;
  size_t dst;
  if (fine_soa) {
    c = i / nsite;
    s = i % nsite;
    dst = (size_t)a * 12 * Vs + (size_t)c * Vs + s;
  } else {
    s = i / dof;
    c = i % dof;
    dst = (size_t)a * nsite * dof + i;
  }
  uint32_t w[4] = {(uint32_t)c, (uint32_t)s, (uint32_t)(alpha0 + a), (uint32_t)lvl};
  philox10(w, k0, k1);
  out[dst] = make_double2((double)(int32_t)w[0] * 0x1p-31, (double)(int32_t)w[1] * 0x1p-31);
}

int start_vectors(long nsite, int dof, uint64_t seed, int lvl, int alpha0, int count, double2 *out, int fine_soa,
                  long Vs, hipStream_t st) {
  dim3 grid((unsigned)((nsite * dof + TB - 1) / TB), count);
  hipLaunchKernelGGL(k_start_vectors, grid, dim3(TB), 0, st, nsite, dof, (uint32_t)seed, (uint32_t)(seed >> 32), lvl,
                     alpha0, out, fine_soa, Vs);
  WMG_HIP(hipGetLastError());
  return 0;
}

// ------------------------------------------------------------ geometry help
struct BlockGeom {
  int L[4], b[4], Lc[4];
  long V, Vc;
  long Vs;  // fine-lattice site stride
  int bs, dof;
  int ns;   // parts of the per-site components: 2 chiralities or 4 spins
};

static BlockGeom make_bg(const Geom &g, int dof, const int b[4], int ns = 2) {
  BlockGeom bg;
  bg.ns = ns;
  for (int i = 0; i < 4; i++) {
    bg.L[i] = g.L[i];
    bg.b[i] = b[i];
    bg.Lc[i] = g.L[i] / b[i];
  }
  bg.V = g.V;
  bg.Vs = g.Vs;
  bg.Vc = (long)bg.Lc[0] * bg.Lc[1] * bg.Lc[2] * bg.Lc[3];
  bg.bs = b[0] * b[1] * b[2] * b[3];
  bg.dof = dof;
  return bg;
}

// fine site of element k of coarse site xh
__device__ __forceinline__ long block_site(const BlockGeom &bg, long xh, int k) {
  int xc[4], x[4];
  site_coords(bg.Lc, xh, xc);
  int w0 = k % bg.b[0], r = k / bg.b[0];
  int w1 = r % bg.b[1]; r /= bg.b[1];
  int w2 = r % bg.b[2]; int w3 = r / bg.b[2];
  x[0] = xc[0] * bg.b[0] + w0;
  x[1] = xc[1] * bg.b[1] + w1;
  x[2] = xc[2] * bg.b[2] + w2;
  x[3] = xc[3] * bg.b[3] + w3;
  return site_index(bg.L, x);
}

// element e -> (k, c)
template <int FINE> __device__ __forceinline__ void elem_kc(const BlockGeom &bg, int e, int &k, int &c) {
  if (FINE) { c = e / bg.bs; k = e % bg.bs; }
  else { k = e / bg.dof; c = e % bg.dof; }
}

// address of component c of site s, rhs r, in a level vector
template <int FINE> __device__ __forceinline__ size_t vec_addr(const BlockGeom &bg, int r, long s, int c) {
  if (FINE) return ((size_t)r * 12 + c) * bg.Vs + s;
  return ((size_t)r * bg.V + s) * bg.dof + c;
}

// workgroup sum of NV complex numbers held per thread; result in sh_out
template <int NV>
__device__ __forceinline__ void wg_csum(cx<double> v[NV], double *sh /* [4][2*NV] */, double *sh_out /* [2*NV] */) {
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
    sh_out[threadIdx.x] = x;
  }
  __syncthreads();
}

// ------------------------------------------------------------ block Gram-Schmidt
// One workgroup per (coarse site, chirality).  The nv vectors are gathered
// into the block-major P slab, then orthonormalised in order, each against
// the already finished ones with classical Gram-Schmidt applied twice (CGS2,
// numerically equivalent to modified GS twice), unit norm, positive real
// diagonal of R.  EPT = elements per thread.
template <int FINE, int EPT>
__global__ void __launch_bounds__(TB) k_block_gs(BlockGeom bg, int a0, int nv, const double2 *__restrict__ vecs,
                                                double2 *__restrict__ P, int *fail) {
  long xh = blockIdx.x;
  int chi = blockIdx.y;
  int h = bg.dof / bg.ns;
  int E = bg.bs * bg.dof;
  __shared__ double sh[4 * 2 * 8];
  __shared__ double red[2 * 8];
  __shared__ double coef[2 * 64];
  // gather: element list of this chirality for this thread
  int my_e[EPT];
  int nmine = 0;
  for (int e = threadIdx.x, q = 0; q < EPT; q++, e += TB) {
    my_e[q] = -1;
    if (e < E) {
      int k, c;
      elem_kc<FINE>(bg, e, k, c);
      if (c / h == chi) my_e[q] = e;
    }
  }
  (void)nmine;
  // vector a depends on vectors 0 .. a-1 only: columns below a0 are kept
  for (int a = a0; a < nv; a++) {
    cx<double> v[EPT];
    double n0loc = 0;
#pragma unroll
    for (int q = 0; q < EPT; q++) {
      v[q] = czero<double>();
      if (my_e[q] >= 0) {
        int k, c;
        elem_kc<FINE>(bg, my_e[q], k, c);
        long s = block_site(bg, xh, k);
        v[q] = ldc(vecs + (FINE ? (size_t)a * 12 * bg.Vs + (size_t)c * bg.Vs + s
                                : (size_t)a * bg.V * bg.dof + (size_t)s * bg.dof + c));
        n0loc += v[q].re * v[q].re + v[q].im * v[q].im;
      }
    }
    {
      cx<double> t[1] = {{n0loc, 0.0}};
      wg_csum<1>(t, sh, red);
    }
    double n0 = red[0];
    for (int pass = 0; pass < 2; pass++) {
      // coefficients <q_j, v> for all j < a, in chunks of 8
      for (int j0 = 0; j0 < a; j0 += 8) {
        cx<double> d[8];
#pragma unroll
        for (int jj = 0; jj < 8; jj++) {
          d[jj] = czero<double>();
          int j = j0 + jj;
          if (j < a) {
#pragma unroll
            for (int q = 0; q < EPT; q++)
              if (my_e[q] >= 0) {
                cx<double> qj = ldc(P + ((size_t)j * bg.Vc + xh) * E + my_e[q]);
                d[jj] = cfmac(qj, v[q], d[jj]);
              }
          }
        }
        wg_csum<8>(d, sh, red);
        if (threadIdx.x < 16 && j0 * 2 + (int)threadIdx.x < 2 * 64) coef[j0 * 2 + threadIdx.x] = red[threadIdx.x];
        __syncthreads();
      }
      for (int j = 0; j < a; j++) {
        cx<double> cj = {coef[2 * j], coef[2 * j + 1]};
#pragma unroll
        for (int q = 0; q < EPT; q++)
          if (my_e[q] >= 0) {
            cx<double> qj = ldc(P + ((size_t)j * bg.Vc + xh) * E + my_e[q]);
            v[q] = v[q] - cj * qj;
          }
      }
      __syncthreads();
    }
    double nl = 0;
#pragma unroll
    for (int q = 0; q < EPT; q++) nl += v[q].re * v[q].re + v[q].im * v[q].im;
    {
      cx<double> t[1] = {{nl, 0.0}};
      wg_csum<1>(t, sh, red);
    }
    double nn = red[0];
    if (!(nn > 1e-24 * n0) || n0 == 0) {
      if (threadIdx.x == 0) atomicOr(fail, 1);
      nn = 1;
    }
    double inv = 1.0 / sqrt(nn);
#pragma unroll
    for (int q = 0; q < EPT; q++)
      if (my_e[q] >= 0) stc(P + ((size_t)a * bg.Vc + xh) * E + my_e[q], inv * v[q]);
    __syncthreads();
  }
}

int block_orthonormalize(const Geom &g, int dof, const int b[4], int nv, const double2 *vecs, int fine_soa, double2 *P,
                         int *fail_dev, hipStream_t st, int ns, int a0) {
  BlockGeom bg = make_bg(g, dof, b, ns);
  int E = bg.bs * dof;
  int ept = (E + TB - 1) / TB;
  if (nv > 64) return set_error(-1, "block_orthonormalize: nv=%d > 64", nv);
  if (a0 < 0 || a0 >= nv) return set_error(-1, "block_orthonormalize: first vector %d of %d", a0, nv);
  if ((ns != 2 && ns != 4) || dof % ns) return set_error(-1, "block_orthonormalize: %d parts of %d", ns, dof);
  dim3 grid((unsigned)bg.Vc, ns);
#define GS_CASE(F, N)                                                                                      \
  if (fine_soa == F && ept <= N) {                                                                        \
    hipLaunchKernelGGL((k_block_gs<F, N>), grid, dim3(TB), 0, st, bg, a0, nv, vecs, P, fail_dev);         \
    WMG_HIP(hipGetLastError());                                                                            \
    return 0;                                                                                              \
  }
  GS_CASE(1, 4) GS_CASE(1, 8) GS_CASE(1, 16) GS_CASE(1, 32)
  GS_CASE(0, 4) GS_CASE(0, 8) GS_CASE(0, 16) GS_CASE(0, 32)
#undef GS_CASE
  return set_error(-1, "block_orthonormalize: block too large (%d elements)", E);
}

// ------------------------------------------------------------ restriction
template <class TP> struct pscale {
  static __device__ __forceinline__ float get(const float *, size_t) { return 1.f; }
};
template <> struct pscale<__half2> {
  static __device__ __forceinline__ float get(const float *s, size_t i) { return s[i]; }
};

// one workgroup per (coarse site, rhs); alpha processed in chunks of 16/NS
// (NS parts of the per-site components)
template <int FINE, int EPT, class TP, class TV, int NS>
__global__ void __launch_bounds__(TB) k_restrict(BlockGeom bg, int nv, const TP *__restrict__ P,
                                                const float *__restrict__ Pscale, const TV *__restrict__ fine,
                                                TV *__restrict__ coarse, int nrhs) {
  using R = typename store_traits<TV>::real;
  // workgroups of one aggregate (all rhs) are adjacent: its P is re-read
  // from cache, not HBM
  long xh = blockIdx.x / nrhs;
  int r = (int)(blockIdx.x % nrhs);
  int E = bg.bs * bg.dof, h = bg.dof / NS;
  // 16 accumulators: ACH null vectors per chunk for each of the NS parts
  constexpr int ACH = 16 / NS;
  const int nc = NS * nv;
  __shared__ double sh[4 * 2 * 16];
  __shared__ double red[2 * 16];
  cx<R> v[EPT];
  int ch[EPT];
  size_t sidx[EPT];
#pragma unroll
  for (int q = 0; q < EPT; q++) {
    int e = threadIdx.x + q * TB;
    v[q] = czero<R>();
    ch[q] = -1;
    if (e < E) {
      int k, c;
      elem_kc<FINE>(bg, e, k, c);
      long s = block_site(bg, xh, k);
      auto t = ldc(fine + vec_addr<FINE>(bg, r, s, c));
      v[q] = {(R)t.re, (R)t.im};
      ch[q] = c / h;
      sidx[q] = (size_t)xh * bg.bs + k;
    }
  }
  for (int a0 = 0; a0 < nv; a0 += ACH) {
    cx<double> acc[16];
#pragma unroll
    for (int j = 0; j < 16; j++) acc[j] = czero<double>();
#pragma unroll
    for (int jj = 0; jj < ACH; jj++) {
      int a = a0 + jj;
      if (a < nv) {
#pragma unroll
        for (int q = 0; q < EPT; q++) {
          if (ch[q] < 0) continue;
          int e = threadIdx.x + q * TB;
          auto p = ldc(P + ((size_t)a * bg.Vc + xh) * E + e);
          float sc = pscale<TP>::get(Pscale, (size_t)a * bg.Vc * bg.bs + sidx[q]);
          cx<R> pv = {(R)(sc * p.re), (R)(sc * p.im)};
          cx<R> t = cmulc(pv, v[q]);
#pragma unroll
          for (int pt = 0; pt < NS; pt++)
            if (pt == ch[q]) acc[pt * ACH + jj] = acc[pt * ACH + jj] + cx<double>{t.re, t.im};
        }
      }
    }
    wg_csum<16>(acc, sh, red);
    if (threadIdx.x < 16) {
      int jj = threadIdx.x % ACH, chi = threadIdx.x / ACH, a = a0 + jj;
      if (chi < NS && a < nv)
        stc(coarse + ((size_t)r * bg.Vc + xh) * nc + chi * nv + a,
            cx<double>{red[2 * threadIdx.x], red[2 * threadIdx.x + 1]});
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ prolongation
// One workgroup per coarse site (XCD-contiguous order).  The coarse values of
// RC right-hand sides are staged in LDS; every thread takes its aggregate
// elements, reads each P entry once and applies it to all RC right-hand
// sides held in registers (one pass over P per chunk of RC).
template <int FINE, int EPT, int RC, class TP, class TV>
__global__ void __launch_bounds__(TB) k_prolong(BlockGeom bg, int nv, const TP *__restrict__ P,
                                               const float *__restrict__ Pscale, const TV *__restrict__ coarse,
                                               TV *__restrict__ fine, int nrhs) {
  using R = typename store_traits<TV>::real;
  long xh = xcd_tile(blockIdx.x, gridDim.x);
  if (xh >= bg.Vc) return;
  const int E = bg.bs * bg.dof, h = bg.dof / bg.ns, n = bg.ns * nv;  // n <= 128
  __shared__ cx<R> cs[RC * 128];
  for (int r0 = 0; r0 < nrhs; r0 += RC) {
    int rc = nrhs - r0 < RC ? nrhs - r0 : RC;
    __syncthreads();
    for (int i = threadIdx.x; i < rc * n; i += TB) {
      int r = i / n, j = i % n;
      auto t = ldc(coarse + ((size_t)(r0 + r) * bg.Vc + xh) * n + j);
      cs[r * n + j] = {(R)t.re, (R)t.im};
    }
    __syncthreads();
#pragma unroll 1
    for (int q = 0; q < EPT; q++) {
      int e = threadIdx.x + q * TB;
      if (e >= E) break;
      int k, c;
      elem_kc<FINE>(bg, e, k, c);
      const int off = (c / h) * nv;
      const size_t si = (size_t)xh * bg.bs + k;
      cx<R> acc[RC];
#pragma unroll
      for (int r = 0; r < RC; r++) acc[r] = czero<R>();
      // P entries (and scales) of 8 null vectors in flight at once
      for (int a0 = 0; a0 < nv; a0 += 8) {
        cx<R> pv[8];
#pragma unroll
        for (int u = 0; u < 8; u++) {
          const int a = a0 + u < nv ? a0 + u : nv - 1;
          auto pv0 = ldc(P + ((size_t)a * bg.Vc + xh) * E + e);
          float sc = pscale<TP>::get(Pscale, (size_t)a * bg.Vc * bg.bs + si);
          pv[u] = {(R)(sc * pv0.re), (R)(sc * pv0.im)};
        }
#pragma unroll
        for (int u = 0; u < 8; u++)
          if (a0 + u < nv)
#pragma unroll
            for (int r = 0; r < RC; r++)
              if (r < rc) acc[r] = cfma(pv[u], cs[r * n + off + a0 + u], acc[r]);
      }
      long s = block_site(bg, xh, k);
#pragma unroll
      for (int r = 0; r < RC; r++)
        if (r < rc) stc(fine + vec_addr<FINE>(bg, r0 + r, s, c), acc[r]);
    }
  }
}

// ------------------------------------------------------------ MFMA restriction
// Fine-level restriction of many right-hand sides on the matrix cores.  Per
// aggregate xh and chirality chi the complex product
//   O[alpha][r] = sum_e conj(P[alpha][e]) v[r][e]      (e: elements of chi)
// is two real GEMMs over the same B = [vr; vi] (K = 2 x elements, N = R):
//   Or = [Pr | Pi] B,   Oi = [-Pi | Pr] B,
// the second A operand read from the same LDS tile of P at the other half
// with a sign.  Streamed in chunks of RCH elements: the chunk of P (FP16
// with its per-site scale, expanded to FP32) and of all R vectors is staged
// in LDS, so P and the vectors are each read once.  Both LDS tiles are kept
// k-contiguous with a row stride of 2*RCH+4 floats, which spreads the 16
// rows x 4 k of an MFMA fragment over all banks.  Fine sites of the block
// come from a per-workgroup offset table (no index arithmetic per element).
typedef float floatx4 __attribute__((ext_vector_type(4)));
// RCH elements per chunk (32, 64 or 128: the autotuner picks; smaller chunks
// take less LDS and allow more resident workgroups, larger ones fewer barriers)
template <int RCH>
__global__ void __launch_bounds__(TB) k_restrict_mfma(BlockGeom bg, int nv, const __half2 *__restrict__ P,
                                                     const float *__restrict__ Pscale, const float2 *__restrict__ fine,
                                                     float2 *__restrict__ coarse, int nrhs) {
  constexpr int RLD = 2 * RCH + 4;  // LDS row stride
  __shared__ float As[32 * RLD];
  __shared__ float Bt[32 * RLD];
  __shared__ int soff[256];  // fine-site offset of block element k from the block's first site
  long xh = xcd_tile(blockIdx.x, gridDim.x);
  if (xh >= bg.Vc) return;
  const long origin = block_site(bg, xh, 0);
  for (int k = threadIdx.x; k < bg.bs; k += TB) soff[k] = (int)(block_site(bg, xh, k) - origin);
  const int r0 = blockIdx.y * 32;
  const int R = nrhs - r0 < 32 ? nrhs - r0 : 32;
  const int E = bg.bs * 12, H = E / bg.ns, nc = bg.ns * nv;
  const int MTr = (nv + 15) / 16, NTr = (R + 15) / 16;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // zero the padding rows once (rows nv..31 of A, columns R..31 of B)
  for (int i = threadIdx.x; i < (32 - nv) * RLD; i += TB) As[nv * RLD + i] = 0.f;
  for (int i = threadIdx.x; i < (32 - R) * RLD; i += TB) Bt[R * RLD + i] = 0.f;
  const int mt = w / 2, nt = w % 2;  // wave w: row tile w/2, rhs tile w%2
  const bool mine = mt < MTr && nt < NTr;
  for (int chi = 0; chi < bg.ns; chi++) {
    floatx4 accr = floatx4{0.f, 0.f, 0.f, 0.f}, acci = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int e0 = 0; e0 < H; e0 += RCH) {
      // the chunk lies inside one spin-colour component c0 (bs % RCH == 0)
      const int g0 = chi * H + e0, c0 = g0 / bg.bs, k0 = g0 % bg.bs;
      __syncthreads();
      for (int i = threadIdx.x; i < nv * RCH; i += TB) {
        int a = i / RCH, e = i % RCH;
        float2 pv = __half22float2(P[((size_t)a * bg.Vc + xh) * E + g0 + e]);
        float sc = Pscale[((size_t)a * bg.Vc + xh) * bg.bs + k0 + e];
        As[a * RLD + e] = sc * pv.x;
        As[a * RLD + RCH + e] = sc * pv.y;
      }
      for (int i = threadIdx.x; i < R * RCH; i += TB) {
        int r = i / RCH, e = i % RCH;
        float2 v = fine[((size_t)(r0 + r) * 12 + c0) * bg.Vs + origin + soff[k0 + e]];
        Bt[r * RLD + e] = v.x;
        Bt[r * RLD + RCH + e] = v.y;
      }
      __syncthreads();
      if (mine) {
        const float *ar = As + (mt * 16 + (lane & 15)) * RLD + (lane >> 4);
        const float *br = Bt + (nt * 16 + (lane & 15)) * RLD + (lane >> 4);
#pragma unroll
        for (int ks = 0; ks < 2 * RCH / 4; ks++) {
          const float b = br[ks * 4];
          const float a2 = ks < RCH / 4 ? -ar[(ks + RCH / 4) * 4] : ar[(ks - RCH / 4) * 4];
          accr = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[ks * 4], b, accr, 0, 0, 0);
          acci = __builtin_amdgcn_mfma_f32_16x16x4f32(a2, b, acci, 0, 0, 0);
        }
      }
    }
    if (mine) {
#pragma unroll
      for (int v = 0; v < 4; v++) {
        int a = mt * 16 + 4 * (lane >> 4) + v, r = nt * 16 + (lane & 15);
        if (a < nv && r < R)
          coarse[((size_t)(r0 + r) * bg.Vc + xh) * nc + chi * nv + a] = make_float2(accr[v], acci[v]);
      }
    }
  }
}

// The same restriction with FP16 products (v_mfma_f32_16x16x16f16, FP32
// accumulation): the P chunk as P16 x scale rounded to FP16, the vectors
// times one power-of-two scale per rhs that brings its 2-norm (rn2, the
// squared norm per rhs at stride rstride) to [1024, 2048), so every entry
// stays below 2048 and the rounding is 2^-11 relative.  Each lane's four
// consecutive k of A and of B (8-byte LDS reads) form one fragment; the
// imaginary part's A = [-Pi | Pr] is read from the same tile at the other
// half with a sign (RCH a multiple of 16: the switch falls between
// fragments).
typedef _Float16 half4 __attribute__((ext_vector_type(4)));
template <int RCH>
__global__ void __launch_bounds__(TB) k_restrict_mfma_h(BlockGeom bg, int nv, const __half2 *__restrict__ P,
                                                       const float *__restrict__ Pscale,
                                                       const float2 *__restrict__ fine, float2 *__restrict__ coarse,
                                                       int nrhs, const double *__restrict__ rn2, int rstride) {
  static_assert(RCH % 16 == 0, "fragments of 16 k");
  constexpr int RLDH = 2 * RCH + 8;  // LDS row stride in halves
  __shared__ _Float16 Ah[32 * RLDH];
  __shared__ _Float16 Bh[32 * RLDH];
  __shared__ int soff[256];
  __shared__ float bsh[32];
  long xh = xcd_tile(blockIdx.x, gridDim.x);
  if (xh >= bg.Vc) return;
  const long origin = block_site(bg, xh, 0);
  for (int k = threadIdx.x; k < bg.bs; k += TB) soff[k] = (int)(block_site(bg, xh, k) - origin);
  const int r0 = blockIdx.y * 32;
  const int R = nrhs - r0 < 32 ? nrhs - r0 : 32;
  if ((int)threadIdx.x < R) {
    const double q = rn2[(size_t)(r0 + threadIdx.x) * rstride];
    int e = 0;
    (void)frexp(sqrt(q > 0 ? q : 0.0), &e);
    const int k = 11 - e < -126 ? -126 : (11 - e > 126 ? 126 : 11 - e);
    bsh[threadIdx.x] = q > 0 ? ldexpf(1.f, k) : 1.f;
  }
  const int E = bg.bs * 12, H = E / bg.ns, nc = bg.ns * nv;
  const int MTr = (nv + 15) / 16, NTr = (R + 15) / 16;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int i = threadIdx.x; i < (32 - nv) * RLDH; i += TB) Ah[nv * RLDH + i] = (_Float16)0.f;
  for (int i = threadIdx.x; i < (32 - R) * RLDH; i += TB) Bh[R * RLDH + i] = (_Float16)0.f;
  const int mt = w / 2, nt = w % 2;
  const bool mine = mt < MTr && nt < NTr;
  const int krow = lane >> 4;
  for (int chi = 0; chi < bg.ns; chi++) {
    floatx4 accr = floatx4{0.f, 0.f, 0.f, 0.f}, acci = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int e0 = 0; e0 < H; e0 += RCH) {
      const int g0 = chi * H + e0, c0 = g0 / bg.bs, k0 = g0 % bg.bs;
      __syncthreads();  // the previous chunk is consumed (and bsh is written)
      for (int i = threadIdx.x; i < nv * RCH; i += TB) {
        int a = i / RCH, e = i % RCH;
        float2 pv = __half22float2(P[((size_t)a * bg.Vc + xh) * E + g0 + e]);
        float sc = Pscale[((size_t)a * bg.Vc + xh) * bg.bs + k0 + e];
        Ah[a * RLDH + e] = (_Float16)(sc * pv.x);
        Ah[a * RLDH + RCH + e] = (_Float16)(sc * pv.y);
      }
      for (int i = threadIdx.x; i < R * RCH; i += TB) {
        int r = i / RCH, e = i % RCH;
        float2 v = fine[((size_t)(r0 + r) * 12 + c0) * bg.Vs + origin + soff[k0 + e]];
        const float bs = bsh[r];
        Bh[r * RLDH + e] = (_Float16)(v.x * bs);
        Bh[r * RLDH + RCH + e] = (_Float16)(v.y * bs);
      }
      __syncthreads();
      if (mine) {
        const _Float16 *ar = Ah + (mt * 16 + (lane & 15)) * RLDH + 4 * krow;
        const _Float16 *br = Bh + (nt * 16 + (lane & 15)) * RLDH + 4 * krow;
#pragma unroll
        for (int b = 0; b < 2 * RCH / 16; b++) {
          half4 a1, a2, bv;
          __builtin_memcpy(&a1, ar + 16 * b, 8);
          __builtin_memcpy(&bv, br + 16 * b, 8);
          if (b < RCH / 16) {
            __builtin_memcpy(&a2, ar + 16 * b + RCH, 8);
            a2 = -a2;
          } else {
            __builtin_memcpy(&a2, ar + 16 * b - RCH, 8);
          }
          accr = __builtin_amdgcn_mfma_f32_16x16x16f16(a1, bv, accr, 0, 0, 0);
          acci = __builtin_amdgcn_mfma_f32_16x16x16f16(a2, bv, acci, 0, 0, 0);
        }
      }
    }
    if (mine) {
      const int r = nt * 16 + (lane & 15);
      const float inv = r < R ? 1.f / bsh[r] : 0.f;
#pragma unroll
      for (int v = 0; v < 4; v++) {
        int a = mt * 16 + 4 * (lane >> 4) + v;
        if (a < nv && r < R)
          coarse[((size_t)(r0 + r) * bg.Vc + xh) * nc + chi * nv + a] = make_float2(accr[v] * inv, acci[v] * inv);
      }
    }
  }
}

// ------------------------------------------------------------ MFMA prolongation
// Fine-level prolongation of many right-hand sides on the matrix cores:
// per aggregate xh and chirality chi, for 16 block elements e at a time,
//   F[r][e] = sum_alpha C[r][alpha] P[alpha][e]
// as two real GEMMs with the right-hand sides as rows (M = R), the elements
// as columns and K = 2 Nv:
//   Fr = [Cr | Ci] [Pr; -Pi],   Fi = [Cr | Ci] [Pi; Pr].
// The coarse values [Cr | Ci] of the aggregate are staged in LDS one
// chirality at a time; each lane loads the P entries of its element column
// straight from HBM (one FP16 complex per alpha, with its per-site scale)
// and forms both B operands from them.  A lane's results are (re, im) pairs
// of 16 consecutive elements, i.e. x-runs of 4 sites, per rhs.  A workgroup
// takes G aggregates adjacent in x, one wave each, which walk their element
// tiles in step; with G = 4 each tile's results go through LDS (two
// barriers per tile, one buffer: the smaller LDS footprint keeps three
// workgroups per CU) and the workgroup writes them as 16-site
// x-runs, whole 128-byte lines of the FP32 output (4-site runs written
// straight from the lanes were fetched before being written: the line was
// read in full for every partial write).
template <int NV, int G>
__global__ void __launch_bounds__(TB) k_prolong_mfma(BlockGeom bg, const __half2 *__restrict__ P,
                                                    const float *__restrict__ Pscale, const float2 *__restrict__ coarse,
                                                    float2 *__restrict__ fine, int nrhs) {
  constexpr int Q = NV / 4;        // k-steps per half of K = 2 NV
  constexpr int LDA = 2 * NV + 4;  // LDS row stride of [Cr | Ci]
  constexpr int NW = TB / 64;      // waves
  __shared__ float Ac[G == 4 ? NW : 1][32 * LDA];  // per aggregate: [Cr | Ci] of one chirality
  __shared__ int soff[256];
  // G = 4: staged results [aggregate][rhs][element] (+1 pad)
  __shared__ float2 Ob[G == 4 ? NW : 1][G == 4 ? 32 : 1][17];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, col = lane & 15, krow = lane >> 4;
  // G = 4: wave w takes aggregate 4 g + w (x-adjacent); G = 1: one aggregate
  // per workgroup, its element tiles spread over the waves
  const long grp = xcd_tile(blockIdx.x, gridDim.x);
  const long xh = G == 4 ? grp * 4 + w : grp;
  const long ngrp = G == 4 ? bg.Vc / 4 : bg.Vc;
  if (grp >= ngrp) return;
  for (int k = threadIdx.x; k < bg.bs; k += TB) soff[k] = (int)(block_site(bg, 0, k) - block_site(bg, 0, 0));
  const long origin = block_site(bg, xh, 0);
  const int r0 = blockIdx.y * 32;
  const int R = nrhs - r0 < 32 ? nrhs - r0 : 32;
  const int NTr = (R + 15) / 16;
  const int E = bg.bs * 12, H = E / bg.ns, nt_el = H / 16, nc = bg.ns * NV;
  float *A = Ac[G == 4 ? w : 0];
  for (int chi = 0; chi < bg.ns; chi++) {
    __syncthreads();  // previous chirality's tiles done
    if (G == 4) {
      for (int i = lane; i < 32 * NV; i += 64) {
        const int r = i / NV, a = i % NV;
        float2 v = make_float2(0.f, 0.f);
        if (r < R) v = coarse[((size_t)(r0 + r) * bg.Vc + xh) * nc + chi * NV + a];
        A[r * LDA + a] = v.x;
        A[r * LDA + NV + a] = v.y;
      }
    } else {
      for (int i = threadIdx.x; i < 32 * NV; i += TB) {
        const int r = i / NV, a = i % NV;
        float2 v = make_float2(0.f, 0.f);
        if (r < R) v = coarse[((size_t)(r0 + r) * bg.Vc + xh) * nc + chi * NV + a];
        A[r * LDA + a] = v.x;
        A[r * LDA + NV + a] = v.y;
      }
    }
    __syncthreads();
    for (int t = G == 4 ? 0 : w; t < nt_el; t += G == 4 ? 1 : NW) {
      const int e0 = chi * H + t * 16;
      const int c = e0 / bg.bs, k0 = e0 % bg.bs;  // 16 elements inside one component (bs % 16 == 0)
      // P entries alpha = 4 ks + krow of element e0 + col
      float pr[Q], pi[Q];
#pragma unroll
      for (int ks = 0; ks < Q; ks++) {
        const int a = 4 * ks + krow;
        const size_t pa = (size_t)a * bg.Vc + xh;
        const float2 pv = __half22float2(P[pa * E + e0 + col]);
        const float sc = Pscale[pa * bg.bs + k0 + col];
        pr[ks] = sc * pv.x;
        pi[ks] = sc * pv.y;
      }
      floatx4 fr[2], fi[2];
#pragma unroll
      for (int m = 0; m < 2; m++) fr[m] = fi[m] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int m = 0; m < 2; m++) {
        if (m >= NTr) break;
        const float *ar = A + (m * 16 + col) * LDA + krow;
#pragma unroll
        for (int ks = 0; ks < 2 * Q; ks++) {
          const float a = ar[4 * ks];
          const float b1 = ks < Q ? pr[ks] : -pi[ks - Q];
          const float b2 = ks < Q ? pi[ks] : pr[ks - Q];
          fr[m] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b1, fr[m], 0, 0, 0);
          fi[m] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b2, fi[m], 0, 0, 0);
        }
      }
      if constexpr (G == 4) {
        __syncthreads();  // the previous tile's results have been written out
#pragma unroll
        for (int m = 0; m < 2; m++) {
          if (m >= NTr) break;
#pragma unroll
          for (int v = 0; v < 4; v++) Ob[w][m * 16 + 4 * krow + v][col] = make_float2(fr[m][v], fi[m][v]);
        }
        __syncthreads();
        // rhs r, block row y (4), x-run of 16 sites over the 4 aggregates
        const long origin0 = origin - (long)w * bg.b[0];
        for (int i = threadIdx.x; i < R * 64; i += TB) {
          const int r = i >> 6, yl = (i >> 4) & 3, xx = i & 15, wa = xx >> 2, el = (xx & 3) + 4 * yl;
          fine[((size_t)(r0 + r) * 12 + c) * bg.Vs + origin0 + (long)wa * bg.b[0] + soff[k0 + el]] = Ob[wa][r][el];
        }
      } else {
        const long site = origin + soff[k0 + col];
#pragma unroll
        for (int m = 0; m < 2; m++) {
          if (m >= NTr) break;
#pragma unroll
          for (int v = 0; v < 4; v++) {
            const int r = m * 16 + 4 * krow + v;
            if (r < R) fine[((size_t)(r0 + r) * 12 + c) * bg.Vs + site] = make_float2(fr[m][v], fi[m][v]);
          }
        }
      }
    }
  }
}

// The same prolongation with FP16 products (v_mfma_f32_16x16x16f16, FP32
// accumulation) for NV a multiple of 8: the coarse values scaled per rhs by
// a power of two (from the partial maxima cpart of their |re|, |im|, as for
// the coarse stencil) and the P entries times their site scale, both rounded
// to FP16; K is ordered as (alpha, re/im) pairs so that each lane's fragment
// holds two alphas' pairs.  The fine field is written in FP32 or, for the
// red/black smoother's residual and last step, in FP16.
// output of the FP16-product prolongation: FP32 or FP16 fine fields
__device__ __forceinline__ void st_fine(float2 *p, float2 v) { *p = v; }
__device__ __forceinline__ void st_fine(__half2 *p, float2 v) { *p = __floats2half2_rn(v.x, v.y); }
template <int NV, int G, class TOUT>
__global__ void __launch_bounds__(TB) k_prolong_mfma_h(BlockGeom bg, const __half2 *__restrict__ P,
                                                      const float *__restrict__ Pscale, const float2 *__restrict__ coarse,
                                                      TOUT *__restrict__ fine, int nrhs,
                                                      const float *__restrict__ cpart) {
  static_assert(NV % 8 == 0, "fragments of four alphas' (re, im) pairs");
  constexpr int NB = NV / 8;        // fragments of 16 k per K = 2 NV
  constexpr int LDA = 2 * NV + 8;   // LDS row stride (halves) of the (re, im)-interleaved coarse values
  constexpr int NW = TB / 64;       // waves
  __shared__ _Float16 Ac[G == 4 ? NW : 1][32 * LDA];  // per aggregate: C of one chirality, scaled per rhs
  __shared__ float bsh[32];                           // per-rhs scale
  __shared__ int soff[256];
  // G = 4: staged results [aggregate][rhs][element] (+1 pad)
  __shared__ float2 Ob[G == 4 ? NW : 1][G == 4 ? 32 : 1][17];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, col = lane & 15, krow = lane >> 4;
  // G = 4: wave w takes aggregate 4 g + w (x-adjacent); G = 1: one aggregate
  // per workgroup, its element tiles spread over the waves
  const long grp = xcd_tile(blockIdx.x, gridDim.x);
  const long xh = G == 4 ? grp * 4 + w : grp;
  const long ngrp = G == 4 ? bg.Vc / 4 : bg.Vc;
  if (grp >= ngrp) return;
  for (int k = threadIdx.x; k < bg.bs; k += TB) soff[k] = (int)(block_site(bg, 0, k) - block_site(bg, 0, 0));
  const long origin = block_site(bg, xh, 0);
  const int r0 = blockIdx.y * 32;
  const int R = nrhs - r0 < 32 ? nrhs - r0 : 32;
  if ((int)threadIdx.x < R) {
    float m = 0.f;
    for (int j = 0; j < COARSE_H_PART; j++) m = fmaxf(m, cpart[(size_t)(r0 + threadIdx.x) * COARSE_H_PART + j]);
    int e = 0;
    (void)frexpf(m, &e);
    const int kx = 11 - e < -126 ? -126 : (11 - e > 126 ? 126 : 11 - e);
    bsh[threadIdx.x] = m > 0.f ? ldexpf(1.f, kx) : 1.f;
  }
  const int NTr = (R + 15) / 16;
  const int E = bg.bs * 12, H = E / bg.ns, nt_el = H / 16, nc = bg.ns * NV;
  _Float16 *A = Ac[G == 4 ? w : 0];
  for (int chi = 0; chi < bg.ns; chi++) {
    __syncthreads();  // previous chirality's tiles done
    if (G == 4) {
      for (int i = lane; i < 32 * NV; i += 64) {
        const int r = i / NV, a = i % NV;
        float2 v = make_float2(0.f, 0.f);
        if (r < R) v = coarse[((size_t)(r0 + r) * bg.Vc + xh) * nc + chi * NV + a];
        const float bs = r < R ? bsh[r] : 0.f;
        A[r * LDA + 2 * a] = (_Float16)(v.x * bs);
        A[r * LDA + 2 * a + 1] = (_Float16)(v.y * bs);
      }
    } else {
      for (int i = threadIdx.x; i < 32 * NV; i += TB) {
        const int r = i / NV, a = i % NV;
        float2 v = make_float2(0.f, 0.f);
        if (r < R) v = coarse[((size_t)(r0 + r) * bg.Vc + xh) * nc + chi * NV + a];
        const float bs = r < R ? bsh[r] : 0.f;
        A[r * LDA + 2 * a] = (_Float16)(v.x * bs);
        A[r * LDA + 2 * a + 1] = (_Float16)(v.y * bs);
      }
    }
    __syncthreads();
    for (int t = G == 4 ? 0 : w; t < nt_el; t += G == 4 ? 1 : NW) {
      const int e0 = chi * H + t * 16;
      const int c = e0 / bg.bs, k0 = e0 % bg.bs;  // 16 elements inside one component (bs % 16 == 0)
      // k slot 16 b + 4 krow + u holds (alpha 8 b + 2 krow + u / 2, re if u
      // even else im) in both operands: the lane's B fragments come from the
      // P entries of two alphas of element e0 + col
      half4 b1[NB], b2[NB];
#pragma unroll
      for (int bb = 0; bb < NB; bb++) {
        float pr[2], pi[2];
#pragma unroll
        for (int u = 0; u < 2; u++) {
          const int a = 8 * bb + 2 * krow + u;
          const size_t pa = (size_t)a * bg.Vc + xh;
          const float2 pv = __half22float2(P[pa * E + e0 + col]);
          const float sc = Pscale[pa * bg.bs + k0 + col];
          pr[u] = sc * pv.x;
          pi[u] = sc * pv.y;
        }
        b1[bb] = half4{(_Float16)pr[0], (_Float16)(-pi[0]), (_Float16)pr[1], (_Float16)(-pi[1])};
        b2[bb] = half4{(_Float16)pi[0], (_Float16)pr[0], (_Float16)pi[1], (_Float16)pr[1]};
      }
      floatx4 fr[2], fi[2];
#pragma unroll
      for (int m = 0; m < 2; m++) fr[m] = fi[m] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int m = 0; m < 2; m++) {
        if (m >= NTr) break;
        const _Float16 *ar = A + (m * 16 + col) * LDA + 4 * krow;
#pragma unroll
        for (int bb = 0; bb < NB; bb++) {
          half4 a;
          __builtin_memcpy(&a, ar + 16 * bb, 8);
          fr[m] = __builtin_amdgcn_mfma_f32_16x16x16f16(a, b1[bb], fr[m], 0, 0, 0);
          fi[m] = __builtin_amdgcn_mfma_f32_16x16x16f16(a, b2[bb], fi[m], 0, 0, 0);
        }
        // undo the rhs scale (rows 4 krow + v of the tile are rhs m 16 + 4 krow + v)
#pragma unroll
        for (int v = 0; v < 4; v++) {
          const int r = m * 16 + 4 * krow + v;
          const float inv = r < R ? 1.f / bsh[r] : 0.f;
          fr[m][v] *= inv;
          fi[m][v] *= inv;
        }
      }
      if constexpr (G == 4) {
        __syncthreads();  // the previous tile's results have been written out
#pragma unroll
        for (int m = 0; m < 2; m++) {
          if (m >= NTr) break;
#pragma unroll
          for (int v = 0; v < 4; v++) Ob[w][m * 16 + 4 * krow + v][col] = make_float2(fr[m][v], fi[m][v]);
        }
        __syncthreads();
        // rhs r, block row y (4), x-run of 16 sites over the 4 aggregates
        const long origin0 = origin - (long)w * bg.b[0];
        for (int i = threadIdx.x; i < R * 64; i += TB) {
          const int r = i >> 6, yl = (i >> 4) & 3, xx = i & 15, wa = xx >> 2, el = (xx & 3) + 4 * yl;
          st_fine(fine + ((size_t)(r0 + r) * 12 + c) * bg.Vs + origin0 + (long)wa * bg.b[0] + soff[k0 + el],
                  Ob[wa][r][el]);
        }
      } else {
        const long site = origin + soff[k0 + col];
#pragma unroll
        for (int m = 0; m < 2; m++) {
          if (m >= NTr) break;
#pragma unroll
          for (int v = 0; v < 4; v++) {
            const int r = m * 16 + 4 * krow + v;
            if (r < R) st_fine(fine + ((size_t)(r0 + r) * 12 + c) * bg.Vs + site, make_float2(fr[m][v], fi[m][v]));
          }
        }
      }
    }
  }
}

template <int FINE, class TP, class TV>
static int launch_transfer(int dir, const BlockGeom &bg, int nv, const void *P, const float *Ps, const void *in,
                           void *out, int nrhs, hipStream_t st) {
  int E = bg.bs * bg.dof;
  int ept = (E + TB - 1) / TB;
  dim3 grid((unsigned)(bg.Vc * nrhs));
#define TR_CASE(N)                                                                                         \
  if (ept <= N) {                                                                                         \
    if (dir == 0 && bg.ns == 4)                                                                            \
      hipLaunchKernelGGL((k_restrict<FINE, N, TP, TV, 4>), grid, dim3(TB), 0, st, bg, nv, (const TP *)P, Ps, \
                         (const TV *)in, (TV *)out, nrhs);                                                 \
    else if (dir == 0)                                                                                     \
      hipLaunchKernelGGL((k_restrict<FINE, N, TP, TV, 2>), grid, dim3(TB), 0, st, bg, nv, (const TP *)P, Ps, \
                         (const TV *)in, (TV *)out, nrhs);                                                 \
    else                                                                                                   \
      hipLaunchKernelGGL((k_prolong<FINE, N, sizeof(TV) == 16 ? 4 : 32, TP, TV>), dim3((unsigned)xcd_grid(bg.Vc)), \
                         dim3(TB), 0, st, bg, nv, (const TP *)P, Ps, (const TV *)in, (TV *)out, nrhs);       \
    WMG_HIP(hipGetLastError());                                                                            \
    return 0;                                                                                              \
  }
  TR_CASE(4) TR_CASE(8) TR_CASE(16) TR_CASE(32)
#undef TR_CASE
  return set_error(-1, "transfer: block too large (%d elements)", E);
}

static int transfer(int dir, const Geom &g, int dof, const int b[4], int nv, int pprec, const void *P,
                    const float *Ps, int vprec, const void *in, void *out, int fine_soa, int nrhs, hipStream_t st,
                    int ns, const double *rn2 = nullptr, int rstride = 0, float *cpart = nullptr,
                    bool out16 = false) {
  BlockGeom bg = make_bg(g, dof, b, ns);
  if (nv > 64) return set_error(-1, "transfer: nv=%d > 64", nv);
  if ((ns != 2 && ns != 4) || dof % ns || ns * nv > 128) return set_error(-1, "transfer: %d parts of %d, nv=%d", ns, dof, nv);
  if (dir == 0 && fine_soa && pprec == P16 && vprec == P32 && nv <= 32 && bg.bs % 32 == 0 && bg.bs <= 256) {
    dim3 grid((unsigned)xcd_grid(bg.Vc), (nrhs + 31) / 32);
    const int chunks[3] = {64, 32, 128};
    int ncand = 0, cand[3];
    for (int c : chunks)
      if (bg.bs % c == 0) cand[ncand++] = c;
    if (rn2) {
      // FP16 products: the chunk size candidates as for the FP32 form
      auto runh = [&](int i) -> int {
        if (cand[i] == 64)
          hipLaunchKernelGGL(k_restrict_mfma_h<64>, grid, dim3(TB), 0, st, bg, nv, (const __half2 *)P, Ps,
                             (const float2 *)in, (float2 *)out, nrhs, rn2, rstride);
        else if (cand[i] == 32)
          hipLaunchKernelGGL(k_restrict_mfma_h<32>, grid, dim3(TB), 0, st, bg, nv, (const __half2 *)P, Ps,
                             (const float2 *)in, (float2 *)out, nrhs, rn2, rstride);
        else
          hipLaunchKernelGGL(k_restrict_mfma_h<128>, grid, dim3(TB), 0, st, bg, nv, (const __half2 *)P, Ps,
                             (const float2 *)in, (float2 *)out, nrhs, rn2, rstride);
        WMG_HIP(hipGetLastError());
        return 0;
      };
      char keyh[160];
      std::snprintf(keyh, sizeof(keyh), "restrict_mfma_h/nv%d-ns%d-bs%d/%dx%dx%dx%d/rhs%d", nv, ns, bg.bs, g.L[0],
                    g.L[1], g.L[2], g.L[3], nrhs);
      int choiceh = 0;
      return tune_choice(keyh, ncand, runh, st, &choiceh);
    }
    auto run = [&](int i) -> int {
      if (cand[i] == 64)
        hipLaunchKernelGGL(k_restrict_mfma<64>, grid, dim3(TB), 0, st, bg, nv, (const __half2 *)P, Ps,
                           (const float2 *)in, (float2 *)out, nrhs);
      else if (cand[i] == 32)
        hipLaunchKernelGGL(k_restrict_mfma<32>, grid, dim3(TB), 0, st, bg, nv, (const __half2 *)P, Ps,
                           (const float2 *)in, (float2 *)out, nrhs);
      else
        hipLaunchKernelGGL(k_restrict_mfma<128>, grid, dim3(TB), 0, st, bg, nv, (const __half2 *)P, Ps,
                           (const float2 *)in, (float2 *)out, nrhs);
      WMG_HIP(hipGetLastError());
      return 0;
    };
    char key[160];
    std::snprintf(key, sizeof(key), "restrict_mfma/nv%d-ns%d-bs%d/%dx%dx%dx%d/rhs%d", nv, ns, bg.bs, g.L[0], g.L[1],
                  g.L[2], g.L[3], nrhs);
    int choice = 0;
    return tune_choice(key, ncand, run, st, &choice);
  }
  if (dir == 1 && fine_soa && pprec == P16 && vprec == P32 && nv % 4 == 0 && nv <= 32 && bg.bs % 16 == 0 &&
      bg.bs <= 256) {
    // four x-adjacent aggregates per workgroup when their 4-site x-runs
    // tile 128-byte lines
    const bool g4 = bg.b[0] == 4 && bg.Lc[0] % 4 == 0;
    dim3 grid((unsigned)xcd_grid(g4 ? bg.Vc / 4 : bg.Vc), (nrhs + 31) / 32);
    if (cpart && nv % 8 == 0) {
      const int rc = rhs_absmax((const float2 *)in, bg.Vc * (long)ns * nv, nrhs, cpart, st);
      if (rc) return rc;
#define PH_CASE(N, TO)                                                                                       \
  if (nv == N) {                                                                                            \
    if (g4)                                                                                                 \
      hipLaunchKernelGGL((k_prolong_mfma_h<N, 4, TO>), grid, dim3(TB), 0, st, bg, (const __half2 *)P, Ps,   \
                         (const float2 *)in, (TO *)out, nrhs, (const float *)cpart);                        \
    else                                                                                                    \
      hipLaunchKernelGGL((k_prolong_mfma_h<N, 1, TO>), grid, dim3(TB), 0, st, bg, (const __half2 *)P, Ps,   \
                         (const float2 *)in, (TO *)out, nrhs, (const float *)cpart);                        \
    WMG_HIP(hipGetLastError());                                                                             \
    return 0;                                                                                               \
  }
      if (out16) {
        PH_CASE(8, __half2) PH_CASE(16, __half2) PH_CASE(24, __half2) PH_CASE(32, __half2)
      } else {
        PH_CASE(8, float2) PH_CASE(16, float2) PH_CASE(24, float2) PH_CASE(32, float2)
      }
#undef PH_CASE
    }
    if (out16) return set_error(-1, "prolong: FP16 output only with FP16 products (Nv a multiple of 8)");
#define PM_CASE(N)                                                                                           \
  if (nv == N) {                                                                                            \
    if (g4)                                                                                                 \
      hipLaunchKernelGGL((k_prolong_mfma<N, 4>), grid, dim3(TB), 0, st, bg, (const __half2 *)P, Ps,         \
                         (const float2 *)in, (float2 *)out, nrhs);                                          \
    else                                                                                                    \
      hipLaunchKernelGGL((k_prolong_mfma<N, 1>), grid, dim3(TB), 0, st, bg, (const __half2 *)P, Ps,         \
                         (const float2 *)in, (float2 *)out, nrhs);                                          \
    WMG_HIP(hipGetLastError());                                                                             \
    return 0;                                                                                               \
  }
    PM_CASE(4) PM_CASE(8) PM_CASE(12) PM_CASE(16) PM_CASE(20) PM_CASE(24) PM_CASE(28) PM_CASE(32)
#undef PM_CASE
  }
#define TP_CASE(F, TPT, TVT, PP, VP)                                                                       \
  if (fine_soa == F && pprec == PP && vprec == VP) return launch_transfer<F, TPT, TVT>(dir, bg, nv, P, Ps, in, out, nrhs, st);
  TP_CASE(1, double2, double2, P64, P64)
  TP_CASE(1, float2, float2, P32, P32)
  TP_CASE(1, __half2, float2, P16, P32)
  TP_CASE(0, double2, double2, P64, P64)
  TP_CASE(0, float2, float2, P32, P32)
  TP_CASE(0, __half2, float2, P16, P32)
#undef TP_CASE
  return set_error(-1, "transfer: unsupported precisions P=%d v=%d", pprec, vprec);
}

int restrict_op(const Geom &g, int dof, const int b[4], int nv, int pprec, const void *P, const float *Pscale,
                int vprec, const void *fine, int fine_soa, void *coarse, int nrhs, hipStream_t st, int ns,
                const double *rn2, int rstride) {
  return transfer(0, g, dof, b, nv, pprec, P, Pscale, vprec, fine, coarse, fine_soa, nrhs, st, ns, rn2, rstride);
}

int prolong_op(const Geom &g, int dof, const int b[4], int nv, int pprec, const void *P, const float *Pscale,
               int vprec, const void *coarse, void *fine, int fine_soa, int nrhs, hipStream_t st, int ns,
               float *cpart, bool out16) {
  if (out16 && !prolong_h_supported(g, dof, b, nv, pprec, vprec, fine_soa, ns))
    return set_error(-1, "prolong: FP16 output not supported for this blocking");
  return transfer(1, g, dof, b, nv, pprec, P, Pscale, vprec, coarse, fine, fine_soa, nrhs, st, ns, nullptr, 0, cpart,
                  out16);
}

bool prolong_h_supported(const Geom &g, int dof, const int b[4], int nv, int pprec, int vprec, int fine_soa, int ns) {
  BlockGeom bg = make_bg(g, dof, b, ns);
  return fine_soa && pprec == P16 && vprec == P32 && nv % 8 == 0 && nv <= 32 && bg.bs % 16 == 0 && bg.bs <= 256 &&
         (ns == 2 || ns == 4) && dof % ns == 0;
}

// ------------------------------------------------------------ P precision
// FP64 -> FP32 copy, or FP64 -> FP16 with one scale per (alpha, xh, k) site.
// count = nv * Vc * bs sites; each has dof components at stride `cstride`
// and site stride `sstride` in element units (fine: cstride = bs, site
// stride 1 inside a block; coarse: cstride 1, site stride dof).
__global__ void k_P_to_half(long nsites, int bs, int dof, int fine, const double2 *__restrict__ P,
                            __half2 *__restrict__ Ph, float *__restrict__ scale) {
  long i = blockIdx.x * (long)TB + threadIdx.x;
  if (i >= nsites) return;
  long blk = i / bs;
  int k = (int)(i % bs);
  size_t base = (size_t)blk * bs * dof;
  double mx = 0;
  for (int c = 0; c < dof; c++) {
    size_t e = base + (fine ? (size_t)c * bs + k : (size_t)k * dof + c);
    double2 v = P[e];
    mx = fmax(mx, fmax(fabs(v.x), fabs(v.y)));
  }
  float sc = mx > 0 ? (float)mx : 1.f;
  scale[i] = sc;
  for (int c = 0; c < dof; c++) {
    size_t e = base + (fine ? (size_t)c * bs + k : (size_t)k * dof + c);
    double2 v = P[e];
    Ph[e] = __floats2half2_rn((float)(v.x / sc), (float)(v.y / sc));
  }
}

__global__ void k_P_to_float(size_t n, const double2 *__restrict__ P, float2 *__restrict__ Pf) {
  size_t i = blockIdx.x * (size_t)TB + threadIdx.x;
  if (i < n) Pf[i] = make_float2((float)P[i].x, (float)P[i].y);
}

int P_convert(long nsites_total, const double2 *P64, int pprec, void *Pout, float *scale, int dof, hipStream_t st) {
  // nsites_total = nv * Vc * bs ; bs passed through `scale == nullptr` path is not needed for FP32
  (void)dof;
  if (pprec == P32) {
    size_t n = (size_t)nsites_total * dof;
    hipLaunchKernelGGL(k_P_to_float, dim3((unsigned)((n + TB - 1) / TB)), dim3(TB), 0, st, n, P64, (float2 *)Pout);
    WMG_HIP(hipGetLastError());
    return 0;
  }
  return set_error(-1, "P_convert: use P_convert_half for FP16");
}

int P_convert_half(long nsites_total, int bs, int dof, int fine, const double2 *P64, __half2 *Ph, float *scale,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_P_to_half, dim3((unsigned)((nsites_total + TB - 1) / TB)), dim3(TB), 0, st, nsites_total, bs,
                     dof, fine, P64, Ph, scale);
  WMG_HIP(hipGetLastError());
  return 0;
}

}  // namespace wmg

namespace wmg {
// block-major P -> level vector layout (fine SoA [nv][12][V] or coarse AoS
// [nv][V][dof]) for copying the prolongator out
__global__ void k_P_to_vec(BlockGeom bg, int nv, int fine, const double2 *__restrict__ P, double2 *__restrict__ vec) {
  size_t E = (size_t)bg.bs * bg.dof;
  size_t i = blockIdx.x * (size_t)TB + threadIdx.x;
  size_t tot = (size_t)nv * bg.Vc * E;
  if (i >= tot) return;
  size_t a = i / (bg.Vc * E);
  long xh = (long)((i / E) % bg.Vc);
  int e = (int)(i % E);
  int k, c;
  if (fine) { c = e / bg.bs; k = e % bg.bs; }
  else { k = e / bg.dof; c = e % bg.dof; }
  long s = block_site(bg, xh, k);
  size_t dst = fine ? (a * 12 + c) * bg.Vs + s : (a * bg.V + s) * bg.dof + c;
  vec[dst] = P[i];
}

int P_block_to_vector(const Geom &g, int dof, const int b[4], int nv, const double2 *P, double2 *vec, int fine_soa,
                      hipStream_t st) {
  BlockGeom bg = make_bg(g, dof, b);
  size_t tot = (size_t)nv * bg.Vc * bg.bs * dof;
  hipLaunchKernelGGL(k_P_to_vec, dim3((unsigned)((tot + TB - 1) / TB)), dim3(TB), 0, st, bg, nv, fine_soa, P, vec);
  WMG_HIP(hipGetLastError());
  return 0;
}
}  // namespace wmg
