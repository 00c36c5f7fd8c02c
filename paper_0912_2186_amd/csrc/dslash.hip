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
//
// Links are stored either whole (9 complex numbers) or, for SU(3) fields,
// as their first two rows (6 complex numbers, the 12-real format of the
// paper's GPU kernels, Table 2): the third row of a special unitary matrix
// is the complex conjugate of the cross product of the first two, and the
// kernel rebuilds it in registers.
#include <cstdio>
#include <type_traits>

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

// L2 budgets (bytes per t-slice of a slab) the autotuner tries; the first is
// the default
static constexpr long SWEEP_BUDGETS[5] = {1L << 20, 1L << 19, 1L << 21, 1L << 18, 1L << 22};

static SweepMap make_sweep(const int L[4], int bytes_per_site, long budget = 1L << 20) {
  // among splits whose t-slice takes at most `budget` bytes of L2, the one
  // with the smallest y/z face fraction (neighbours outside the slab); the
  // largest cross-section breaks ties.  If none fits, the smallest
  // cross-section.
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

// third row of an SU(3) matrix from its first two: conj(row0 x row1)
template <class R> __device__ __forceinline__ void su3_third_row(cx<R> u[9]) {
  const cx<R> c0 = u[1] * u[5] - u[2] * u[4];
  const cx<R> c1 = u[2] * u[3] - u[0] * u[5];
  const cx<R> c2 = u[0] * u[4] - u[1] * u[3];
  u[6] = {c0.re, -c0.im};
  u[7] = {c1.re, -c1.im};
  u[8] = {c2.re, -c2.im};
}

// the four spins of one colour (consecutive elements)
__device__ __forceinline__ void ld4(const __half2 *p, cx<float> o[4]) {
  const uint4 v = *(const uint4 *)p;
  const unsigned w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int i = 0; i < 4; i++) {
    __half2 h;
    __builtin_memcpy(&h, &w[i], 4);
    const float2 f = __half22float2(h);
    o[i] = {f.x, f.y};
  }
}
__device__ __forceinline__ void ld4(const float2 *p, cx<float> o[4]) {
  const float4 a = *(const float4 *)p, b = *(const float4 *)(p + 2);
  o[0] = {a.x, a.y};
  o[1] = {a.z, a.w};
  o[2] = {b.x, b.y};
  o[3] = {b.z, b.w};
}
__device__ __forceinline__ void ld4(const double2 *p, cx<double> o[4]) {
#pragma unroll
  for (int i = 0; i < 4; i++) o[i] = ldc(p + i);
}
__device__ __forceinline__ void st4(__half2 *p, const cx<float> o[4]) {
  unsigned w[4];
#pragma unroll
  for (int i = 0; i < 4; i++) {
    const __half2 h = __floats2half2_rn(o[i].re, o[i].im);
    __builtin_memcpy(&w[i], &h, 4);
  }
  *(uint4 *)p = make_uint4(w[0], w[1], w[2], w[3]);
}
__device__ __forceinline__ void st4(float2 *p, const cx<float> o[4]) {
  *(float4 *)p = make_float4(o[0].re, o[0].im, o[1].re, o[1].im);
  *(float4 *)(p + 2) = make_float4(o[2].re, o[2].im, o[3].re, o[3].im);
}
__device__ __forceinline__ void st4(double2 *p, const cx<double> o[4]) {
#pragma unroll
  for (int i = 0; i < 4; i++) stc(p + i, o[i]);
}
// the same with the non-temporal hint (data used once: the line is not
// kept in the caches at the expense of data that is reused)
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void ld4_nt(const __half2 *p, cx<float> o[4]) {
  const u32x4 v = __builtin_nontemporal_load((const u32x4 *)p);
  const unsigned w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int i = 0; i < 4; i++) {
    __half2 h;
    __builtin_memcpy(&h, &w[i], 4);
    const float2 f = __half22float2(h);
    o[i] = {f.x, f.y};
  }
}
__device__ __forceinline__ void ld4_nt(const float2 *p, cx<float> o[4]) { ld4(p, o); }
__device__ __forceinline__ void ld4_nt(const double2 *p, cx<double> o[4]) { ld4(p, o); }
__device__ __forceinline__ void st4_nt(__half2 *p, const cx<float> o[4]) {
  unsigned w[4];
#pragma unroll
  for (int i = 0; i < 4; i++) {
    const __half2 h = __floats2half2_rn(o[i].re, o[i].im);
    __builtin_memcpy(&w[i], &h, 4);
  }
  const u32x4 v = {w[0], w[1], w[2], w[3]};
  __builtin_nontemporal_store(v, (u32x4 *)p);
}
__device__ __forceinline__ void st4_nt(float2 *p, const cx<float> o[4]) { st4(p, o); }
__device__ __forceinline__ void st4_nt(double2 *p, const cx<double> o[4]) { st4(p, o); }
// p[0] = b[0] + lo, p[1] = b[1] + hi, b an FP16 full-lattice component
__device__ __forceinline__ void set_pair_base(float2 *p, const __half2 *b, cx<float> lo, cx<float> hi) {
  const uint2 w = *(const uint2 *)b;
  __half2 h0, h1;
  __builtin_memcpy(&h0, &w.x, 4);
  __builtin_memcpy(&h1, &w.y, 4);
  const float2 f0 = __half22float2(h0), f1 = __half22float2(h1);
  *(float4 *)p = make_float4(f0.x + lo.re, f0.y + lo.im, f1.x + hi.re, f1.y + hi.im);
}
// the same with the pair stored in FP16 (sums formed in FP32, rounded once)
__device__ __forceinline__ void set_pair_base(__half2 *p, const __half2 *b, cx<float> lo, cx<float> hi) {
  const uint2 w = *(const uint2 *)b;
  __half2 h0, h1;
  __builtin_memcpy(&h0, &w.x, 4);
  __builtin_memcpy(&h1, &w.y, 4);
  const float2 f0 = __half22float2(h0), f1 = __half22float2(h1);
  h0 = __floats2half2_rn(f0.x + lo.re, f0.y + lo.im);
  h1 = __floats2half2_rn(f1.x + hi.re, f1.y + hi.im);
  uint2 o;
  __builtin_memcpy(&o.x, &h0, 4);
  __builtin_memcpy(&o.y, &h1, 4);
  *(uint2 *)p = o;
}
__device__ __forceinline__ void set_pair_base(double2 *, const __half2 *, cx<double>, cx<double>) {}
// p[0] += lo, p[1] += hi (two adjacent sites of a full-lattice component)
__device__ __forceinline__ void add_pair(float2 *p, cx<float> lo, cx<float> hi) {
  float4 v = *(float4 *)p;
  *(float4 *)p = make_float4(v.x + lo.re, v.y + lo.im, v.z + hi.re, v.w + hi.im);
}
__device__ __forceinline__ void add_pair(double2 *p, cx<double> lo, cx<double> hi) {
  const double2 a = p[0], b = p[1];
  p[0] = make_double2(a.x + lo.re, a.y + lo.im);
  p[1] = make_double2(b.x + hi.re, b.y + hi.im);
}

// ---------------------------------------------------------------- packed FP16
// Packed half-precision arithmetic of the all-FP16 hopping terms: two FP16
// values per lane and instruction, the complex broadcasts, swaps and signs
// folded into the operands' modifiers (a complex multiply-add is two packed
// FMAs); the FP16 -> FP32 conversion of a term is folded into its FP32
// accumulation through a multiplier `one` the compiler cannot see.
typedef _Float16 h2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ h2 pk_i(h2 a) { return (h2){-a.y, a.x}; }   // i a
__device__ __forceinline__ h2 pk_mi(h2 a) { return (h2){a.y, -a.x}; }  // -i a
// c + a b and c + conj(a) b
__device__ __forceinline__ h2 pk_cfma(h2 a, h2 b, h2 c) {
  const h2 t = __builtin_elementwise_fma(a.xx, b, c);
  return __builtin_elementwise_fma((h2){-a.y, a.y}, b.yx, t);
}
__device__ __forceinline__ h2 pk_cfmac(h2 a, h2 b, h2 c) {
  const h2 t = __builtin_elementwise_fma(a.xx, b, c);
  return __builtin_elementwise_fma((h2){a.y, -a.y}, b.yx, t);
}
__device__ __forceinline__ h2 pk_cmul(h2 a, h2 b) { return __builtin_elementwise_fma((h2){-a.y, a.y}, b.yx, a.xx * b); }
__device__ __forceinline__ h2 pk_ld(const __half2 *p) {
  const unsigned w = *(const unsigned *)p;
  h2 r;
  __builtin_memcpy(&r, &w, 4);
  return r;
}
template <int NR>
__device__ __forceinline__ void pk_link(const __half2 *Up, int mu, unsigned site, int Vs, h2 u[9]) {
#pragma unroll
  for (int e = 0; e < NR; e++) u[e] = pk_ld(Up + (size_t)(mu * NR + e) * Vs + site);
  if (NR == 6) {
    // third row conj(row0 x row1), conj(a b) - conj(c d) as four packed FMAs
    auto cc = [](h2 a, h2 b, h2 c, h2 d) {
      h2 t = a.xx * (h2){b.x, -b.y};
      t = __builtin_elementwise_fma((h2){-a.y, -a.y}, b.yx, t);
      t = __builtin_elementwise_fma(-c.xx, (h2){d.x, -d.y}, t);
      return __builtin_elementwise_fma((h2){c.y, c.y}, d.yx, t);
    };
    u[6] = cc(u[1], u[5], u[2], u[4]);
    u[7] = cc(u[2], u[3], u[0], u[5]);
    u[8] = cc(u[0], u[4], u[1], u[3]);
  }
}
// one colour of the projection from the four stored spins (as proj_pair)
template <int MU, int S>
__device__ __forceinline__ void pk_proj_q(const h2 q[4], h2 &h0, h2 &h1) {
  h2 a0, a1;  // A_mu p_down
  if (MU == 0) { a0 = pk_mi(q[3]); a1 = pk_mi(q[2]); }
  if (MU == 1) { a0 = -q[3]; a1 = q[2]; }
  if (MU == 2) { a0 = pk_mi(q[2]); a1 = pk_i(q[3]); }
  if (MU == 3) { a0 = q[2]; a1 = q[3]; }
  if (S > 0) { h0 = q[0] - a0; h1 = q[1] - a1; }
  else { h0 = q[0] + a0; h1 = q[1] + a1; }
}
// the same from the four spins stored together (half-lattice layout)
template <int MU, int S>
__device__ __forceinline__ void pk_proj(const __half2 *p, h2 &h0, h2 &h1) {
  const uint4 v = *(const uint4 *)p;
  const unsigned w[4] = {v.x, v.y, v.z, v.w};
  h2 q[4];
#pragma unroll
  for (int i = 0; i < 4; i++) __builtin_memcpy(&q[i], &w[i], 4);
  pk_proj_q<MU, S>(q, h0, h1);
}
__device__ __forceinline__ void pk_acc(cx<float> &acc, h2 x, float one) {
  acc.re = __builtin_fmaf((float)x.x, one, acc.re);
  acc.im = __builtin_fmaf((float)x.y, one, acc.im);
}
// upper spins += gf + gb, lower spins += A_mu^dag (gb - gf): the forward and
// backward terms of reconstruct<MU, +1> and reconstruct<MU, -1> together
template <int MU>
__device__ __forceinline__ void pk_recon(const h2 gf[6], const h2 gb[6], cx<float> acc[12], float one) {
#pragma unroll
  for (int c = 0; c < 3; c++) {
    pk_acc(acc[c], gf[c] + gb[c], one);
    pk_acc(acc[3 + c], gf[3 + c] + gb[3 + c], one);
    const h2 d0 = gb[c] - gf[c], d1 = gb[3 + c] - gf[3 + c];
    h2 b0, b1;
    if (MU == 0) { b0 = pk_i(d1); b1 = pk_i(d0); }
    if (MU == 1) { b0 = d1; b1 = -d0; }
    if (MU == 2) { b0 = pk_i(d0); b1 = pk_mi(d1); }
    if (MU == 3) { b0 = d0; b1 = d1; }
    pk_acc(acc[6 + c], b0, one);
    pk_acc(acc[9 + c], b1, one);
  }
}

// ---------------------------------------------------------------- SoA
// Optional fusions for the smoother: bsub != nullptr gives out = bsub - D in
// (residual); RED != 0 also reduces <out, in> and |out|^2 over the
// workgroup into red[(rhs * gridDim.x + block) * 3 + 0..2] for a
// fixed-order finalisation by k_dslash_red_finalize.
// With EO, the output goes to the two half-lattice arrays out (even sites)
// and out_odd (odd sites) in their [rhs][colour][Vhs][spin] layout instead.
template <class TL, class TS, class TO, int RT, int RED, int NR, int EO = 0, class TB = TS>
__global__ void __launch_bounds__(256) k_wilson_soa(const TL *__restrict__ U, const TS *__restrict__ in,
                                                   TO *__restrict__ out, int L0, int L1, int L2, int L3, long V,
                                                   float diagf, double diagd, int nrhs, SweepMap sm, long Vs,
                                                   const TB *__restrict__ bsub, const double *__restrict__ bnrm2,
                                                   int bstride, double *__restrict__ red, int inner,
                                                   float2 *__restrict__ out32, TO *__restrict__ out_odd, long Vhs,
                                                   float one, const float2 *__restrict__ dotv) {
  using R = typename store_traits<TS>::real;
  const R diag = sizeof(R) == 8 ? (R)diagd : (R)diagf;
  // one sweep over the lattice per tile of RT right-hand sides (grid.y)
  const int L[4] = {L0, L1, L2, L3};
  int x[4];
  long s = 0;
  // site-tile workgroup index tb and first rhs r0: grid (tiles, rhs tiles)
  // when inner = 0; else one dimension in which each XCD (blockIdx % 8)
  // sweeps its range of site tiles once per group of `inner` rhs tiles, the
  // group's rhs tiles of one site tile back to back (the last group may be
  // short).  One group of all rhs tiles reads the links once; smaller groups
  // bring the t-neighbours of a tile closer in the XCD's sequence.
  long tb = blockIdx.x;
  int r0 = blockIdx.y * RT;
  if (inner) {
    const int nrt = (nrhs + RT - 1) / RT;
    const long q = (long)blockIdx.x / NXCD;
    const long span = sm.per_xcd * inner;  // blocks of one full group on an XCD
    const int g0 = (int)(q / span) * inner;
    const int gc = min(inner, nrt - g0);
    const long rem = q - (q / span) * span;
    tb = (rem / gc) * NXCD + blockIdx.x % NXCD;
    r0 = (g0 + (int)(rem % gc)) * RT;
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
    for (int e = 0; e < NR; e++) {
      auto v = ldc(U + ((size_t)(mu * NR + e)) * Vs + site);
      u[e] = {(R)v.re, (R)v.im};
    }
    if (NR == 6) su3_third_row(u);
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
  // FP16 links and spinors: projection, SU(3) products and the sum and
  // difference of each direction's forward and backward terms in packed
  // FP16, the directions summed in FP32 (as in the packed red/black hop)
#define WILSON_DIR_PK(MU)                                                                      \
  {                                                                                            \
    long fw = x[MU] == L[MU] - 1 ? s - (long)(L[MU] - 1) * stride[MU] : s + stride[MU];        \
    long bw = x[MU] == 0 ? s + (long)(L[MU] - 1) * stride[MU] : s - stride[MU];                \
    int yf[4] = {x[0], x[1], x[2], x[3]}, yb[4] = {x[0], x[1], x[2], x[3]};                    \
    yf[MU] = x[MU] == L[MU] - 1 ? 0 : x[MU] + 1;                                               \
    yb[MU] = x[MU] == 0 ? L[MU] - 1 : x[MU] - 1;                                               \
    const int lf = local_of(yf), lb = local_of(yb);                                            \
    h2 uf[9], ub[9];                                                                           \
    pk_link<NR>((const __half2 *)U, MU, (unsigned)s, (int)Vs, uf);                             \
    pk_link<NR>((const __half2 *)U, MU, (unsigned)bw, (int)Vs, ub);                            \
    _Pragma("unroll") for (int t = 0; t < RT; t++) {                                           \
      if (r0 + t < nrhs) {                                                                     \
        h2 hh[6], gf[6], gb[6];                                                                \
        _Pragma("unroll") for (int c = 0; c < 3; c++) {                                        \
          h2 q[4];                                                                             \
          _Pragma("unroll") for (int sp = 0; sp < 4; sp++)                                     \
            q[sp] = pk_ld(lf >= 0 ? (const __half2 *)Sh + (t * 12 + sp * 3 + c) * 256 + lf     \
                                  : (const __half2 *)in + ((size_t)(r0 + t) * 12 + sp * 3 + c) * Vs + fw); \
          pk_proj_q<MU, 1>(q, hh[c], hh[3 + c]);                                               \
        }                                                                                      \
        _Pragma("unroll") for (int sp = 0; sp < 2; sp++)                                       \
        _Pragma("unroll") for (int a = 0; a < 3; a++) {                                        \
          h2 v = pk_cmul(uf[3 * a], hh[3 * sp]);                                               \
          v = pk_cfma(uf[3 * a + 1], hh[3 * sp + 1], v);                                       \
          gf[3 * sp + a] = pk_cfma(uf[3 * a + 2], hh[3 * sp + 2], v);                          \
        }                                                                                      \
        _Pragma("unroll") for (int c = 0; c < 3; c++) {                                        \
          h2 q[4];                                                                             \
          _Pragma("unroll") for (int sp = 0; sp < 4; sp++)                                     \
            q[sp] = pk_ld(lb >= 0 ? (const __half2 *)Sh + (t * 12 + sp * 3 + c) * 256 + lb     \
                                  : (const __half2 *)in + ((size_t)(r0 + t) * 12 + sp * 3 + c) * Vs + bw); \
          pk_proj_q<MU, -1>(q, hh[c], hh[3 + c]);                                              \
        }                                                                                      \
        _Pragma("unroll") for (int sp = 0; sp < 2; sp++)                                       \
        _Pragma("unroll") for (int a = 0; a < 3; a++) {                                        \
          h2 v = pk_cfmac(ub[a], hh[3 * sp], (h2){0, 0});                                      \
          v = pk_cfmac(ub[3 + a], hh[3 * sp + 1], v);                                          \
          gb[3 * sp + a] = pk_cfmac(ub[6 + a], hh[3 * sp + 2], v);                             \
        }                                                                                      \
        pk_recon<MU>(gf, gb, acc[t], one);                                                     \
      }                                                                                        \
    }                                                                                          \
  }
  if constexpr (std::is_same<TL, __half2>::value && std::is_same<TS, __half2>::value) {
    WILSON_DIR_PK(0)
    WILSON_DIR_PK(1)
    WILSON_DIR_PK(2)
    WILSON_DIR_PK(3)
  } else {
    WILSON_DIR(0)
    WILSON_DIR(1)
    WILSON_DIR(2)
    WILSON_DIR(3)
  }
#undef WILSON_DIR_PK
#undef WILSON_DIR

#pragma unroll
  for (int t = 0; t < RT; t++) {
    if (r0 + t >= nrhs) continue;
    cx<R> oo[EO ? 12 : 1];
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
      if constexpr (EO) oo[c] = o;
      else if (out) stc(out + ((size_t)(r0 + t) * 12 + c) * Vs + s, o);
      if (out32) stc(out32 + ((size_t)(r0 + t) * 12 + c) * Vs + s, o);
      if (RED) o = as_stored(out, o);
      if (RED) {
        // <out, in> (or <out, dotv> with a partner field) and |out|^2
        cx<R> q = p[c];
        if (dotv) {
          const float2 d = dotv[((size_t)(r0 + t) * 12 + c) * Vs + s];
          q = {(R)d.x, (R)d.y};
        }
        rs[t][0] += (double)o.re * q.re + (double)o.im * q.im;
        rs[t][1] += (double)o.re * q.im - (double)o.im * q.re;
        rs[t][2] += (double)o.re * o.re + (double)o.im * o.im;
      }
    }
    if constexpr (EO) {
      TO *dst = ((x[0] + x[1] + x[2] + x[3]) & 1) ? out_odd : out;
#pragma unroll
      for (int c = 0; c < 3; c++) {
        const cx<R> q4[4] = {oo[c], oo[3 + c], oo[6 + c], oo[9 + c]};
        st4(dst + (((size_t)(r0 + t) * 3 + c) * Vhs + (s >> 1)) * 4, q4);
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

template <class TL, class TS, class TO = TS, int NR = 9, class TB = TS>
static int launch_soa(const Geom &g, const void *U, double m, const void *in, void *out, int nrhs, const void *bsub,
                      double *red, double *red_out, int red_stride, hipStream_t st, const double *bnrm2 = nullptr,
                      int bstride = 0, void *out32 = nullptr, void *out_odd = nullptr, const float2 *dotv = nullptr) {
  if (out_odd && (red || g.L[0] % 2)) return set_error(-1, "wilson_soa: half-lattice output without reductions only");
  const long Vhs = fine_stride(g.V / 2);
  constexpr int RT = sizeof(TS) == 16 ? 1 : 2;
  const int nrt = (nrhs + RT - 1) / RT;
  // Default order: FP64 and FP32 links (288-576 B per site) would be re-read
  // from HBM by every rhs tile's sweep, so the rhs tiles of one site tile
  // run back to back on one XCD and share the links in its L2 (FP64, 28 rhs:
  // 14.6 -> 10.4 ms on 32^3x64); FP16 links are cheap to re-read, and one
  // sweep per rhs tile keeps the spinor halo in L2.  The autotuner also
  // tries the other order and other slab sizes.
  const int inner0 = sizeof(TL) >= 8 && nrt > 1 ? nrt : 0;
  // bytes a site brings into L2 during one sweep: its links and RT spinors
  const int bps = 4 * NR * (int)sizeof(TL) + 24 * (int)sizeof(TS) / 2 * RT;
  const size_t lds = (size_t)(nrhs < RT ? nrhs : RT) * 12 * 256 * sizeof(TS);
  constexpr int NB = (int)(sizeof(SWEEP_BUDGETS) / sizeof(SWEEP_BUDGETS[0]));
  // candidates: every slab budget with the default order, then with the
  // other of (one sweep per rhs tile, all rhs tiles of a site tile back to
  // back), then with groups of 4, 3 and 2 rhs tiles
  int cb[6 * NB], cg[6 * NB], ncand = 0;
  for (int k = 0; k < NB; k++) cb[ncand] = k, cg[ncand++] = inner0;
  if (nrt > 1) {
    for (int k = 0; k < NB; k++) cb[ncand] = k, cg[ncand++] = inner0 ? 0 : nrt;
    for (int gs : {4, 3, 2})
      if (gs < nrt)
        for (int k = 0; k < NB; k++) cb[ncand] = k, cg[ncand++] = gs;
  }
  auto run = [&](int cand) -> int {
    const long budget = SWEEP_BUDGETS[cb[cand]];
    const int inner = cg[cand];
    SweepMap sm = make_sweep(g.L, bps, budget);
    dim3 grid = inner ? dim3((unsigned)(sm.nblocks * nrt)) : dim3((unsigned)sm.nblocks, nrt);
    if (red) {
      hipLaunchKernelGGL((k_wilson_soa<TL, TS, TO, RT, 1, NR, 0, TB>), grid, dim3(256), lds, st, (const TL *)U,
                         (const TS *)in, (TO *)out, g.L[0], g.L[1], g.L[2], g.L[3], g.V, (float)(4.0 + m), 4.0 + m,
                         nrhs, sm, g.Vs, (const TB *)bsub, bnrm2, bstride, red, inner, (float2 *)out32, (TO *)nullptr,
                         Vhs, 1.0f, dotv);
      hipLaunchKernelGGL(k_dslash_red_finalize, dim3(nrhs), dim3(256), 0, st, red, (long)sm.nblocks, red_out,
                         red_stride);
    } else if (out_odd) {
      // instantiated for the smoother's residual forms only (FP32 or FP16
      // input, FP32 bsub)
      if constexpr (std::is_same<TO, __half2>::value && std::is_same<TB, float2>::value)
        hipLaunchKernelGGL((k_wilson_soa<TL, TS, TO, RT, 0, NR, 1, TB>), grid, dim3(256), lds, st, (const TL *)U,
                           (const TS *)in, (TO *)out, g.L[0], g.L[1], g.L[2], g.L[3], g.V, (float)(4.0 + m), 4.0 + m,
                           nrhs, sm, g.Vs, (const TB *)bsub, bnrm2, bstride, (double *)nullptr, inner,
                           (float2 *)out32, (TO *)out_odd, Vhs, 1.0f, (const float2 *)nullptr);
      else
        return set_error(-1, "wilson_soa: half-lattice output not instantiated for these precisions");
    } else {
      hipLaunchKernelGGL((k_wilson_soa<TL, TS, TO, RT, 0, NR, 0, TB>), grid, dim3(256), lds, st, (const TL *)U,
                         (const TS *)in, (TO *)out, g.L[0], g.L[1], g.L[2], g.L[3], g.V, (float)(4.0 + m), 4.0 + m,
                         nrhs, sm, g.Vs, (const TB *)bsub, bnrm2, bstride, (double *)nullptr, inner, (float2 *)out32,
                         (TO *)nullptr, Vhs, 1.0f, (const float2 *)nullptr);
    }
    WMG_HIP(hipGetLastError());
    return 0;
  };
  char key[256];
  std::snprintf(key, sizeof(key), "dslash/l%zu-s%zu-o%zu-nr%d-red%d-b%d-f%d-eo%d/%dx%dx%dx%d/rhs%d", sizeof(TL),
                sizeof(TS), sizeof(TO), NR, red ? (dotv ? 2 : 1) : 0, bsub ? (int)sizeof(TB) : 0, out32 ? 1 : 0,
                out_odd ? 1 : 0,
                g.L[0], g.L[1], g.L[2], g.L[3], nrhs);
  int choice = 0;
  return tune_choice(key, ncand, run, st, &choice);
}

long wilson_red_blocks(const Geom &g) {
  // every (link, spinor) storage pair launch_soa instantiates, links whole
  // (36 complex per site) or compressed (24)
  const int lb[5] = {16, 8, 4, 4, 8}, sb[5] = {24 * 8, 24 * 4 * 2, 24 * 4 * 2, 24 * 2 * 2, 24 * 2 * 2};
  long m = 0;
  for (int i = 0; i < 5; i++)
    for (int nl : {36, 24})
      for (long budget : SWEEP_BUDGETS) {
        long nb = make_sweep(g.L, nl * lb[i] + sb[i], budget).nblocks;
        m = nb > m ? nb : m;
      }
  if (g.L[0] % 2 == 0) {
    const long et = eo_red_tiles(g);
    m = et > m ? et : m;
  }
  return m;
}

int wilson_soa_fused(const Geom &g, int lprec, const void *U, int sprec, double m, const void *in, void *out, int nrhs,
                     const void *bsub, double *red, double *red_out, int red_stride, hipStream_t st, void *out32) {
  if (out32 && sprec != P64) return set_error(-1, "wilson_soa: FP32 copy of the output only for FP64 spinors");
  if (!out && !out32) return set_error(-1, "wilson_soa: no output");
  const bool c12 = (lprec & LK12) != 0;
  const int lp = lprec & ~LK12;
#define WS_LAUNCH(TL, TS, ...)                                                                                  \
  return c12 ? launch_soa<TL, TS, TS, 6>(g, U, m, in, out, nrhs, bsub, red, red_out, red_stride, st, __VA_ARGS__) \
             : launch_soa<TL, TS, TS, 9>(g, U, m, in, out, nrhs, bsub, red, red_out, red_stride, st, __VA_ARGS__)
  if (sprec == P64 && lp == P64) WS_LAUNCH(double2, double2, nullptr, 0, out32);
  if (sprec == P32 && lp == P32) WS_LAUNCH(float2, float2, nullptr, 0, nullptr);
  if (sprec == P32 && lp == P16) WS_LAUNCH(__half2, float2, nullptr, 0, nullptr);
#undef WS_LAUNCH
  return set_error(-1, "wilson_soa: unsupported precision pair link=%d spinor=%d", lp, sprec);
}

int wilson_soa_in16(const Geom &g, int lprec, const void *U, double m, const void *in, void *out, int nrhs,
                    hipStream_t st, double *red, double *red_out, int red_stride, const void *dotv) {
  const bool c12 = (lprec & LK12) != 0;
  if ((lprec & ~LK12) != P32) return set_error(-1, "wilson_soa_in16: FP32 links only");
  if (dotv && !red) return set_error(-1, "wilson_soa_in16: a dot partner needs the reductions");
  return c12 ? launch_soa<float2, __half2, float2, 6>(g, U, m, in, out, nrhs, nullptr, red, red_out, red_stride, st,
                                                      nullptr, 0, nullptr, nullptr, (const float2 *)dotv)
             : launch_soa<float2, __half2, float2, 9>(g, U, m, in, out, nrhs, nullptr, red, red_out, red_stride, st,
                                                      nullptr, 0, nullptr, nullptr, (const float2 *)dotv);
}

int wilson_soa_h16(const Geom &g, const void *U16, int iprec, double m, const void *in, void *out, int nrhs,
                   const void *bsub, const double *bnrm2, int bstride, double *red, double *red_out, int red_stride,
                   hipStream_t st, int lflags, void *out_odd) {
  const bool c12 = (lflags & LK12) != 0;
  if (iprec == P32)
    return c12 ? launch_soa<__half2, float2, __half2, 6>(g, U16, m, in, out, nrhs, bsub, red, red_out, red_stride, st,
                                                         bnrm2, bstride, nullptr, out_odd)
               : launch_soa<__half2, float2, __half2, 9>(g, U16, m, in, out, nrhs, bsub, red, red_out, red_stride, st,
                                                         bnrm2, bstride, nullptr, out_odd);
  if (iprec == P16 && bsub && out_odd)
    return c12 ? launch_soa<__half2, __half2, __half2, 6, float2>(g, U16, m, in, out, nrhs, bsub, red, red_out,
                                                                  red_stride, st, bnrm2, bstride, nullptr, out_odd)
               : launch_soa<__half2, __half2, __half2, 9, float2>(g, U16, m, in, out, nrhs, bsub, red, red_out,
                                                                  red_stride, st, bnrm2, bstride, nullptr, out_odd);
  if (out_odd) return set_error(-1, "wilson_soa_h16: half-lattice output only with FP32 bsub");
  if (iprec == P16 && !bsub)
    return c12 ? launch_soa<__half2, __half2, __half2, 6>(g, U16, m, in, out, nrhs, nullptr, red, red_out, red_stride,
                                                          st)
               : launch_soa<__half2, __half2, __half2, 9>(g, U16, m, in, out, nrhs, nullptr, red, red_out, red_stride,
                                                          st);
  return set_error(-1, "wilson_soa_h16: input precision %d%s", iprec, bsub ? " with bsub" : "");
}

int wilson_soa(const Geom &g, int lprec, const void *U, int sprec, double m, const void *in, void *out, int nrhs,
               hipStream_t st) {
  return wilson_soa_fused(g, lprec, U, sprec, m, in, out, nrhs, nullptr, nullptr, nullptr, 0, st);
}

// ---------------------------------------------------------------- red/black
// Even-odd decomposition (Sec. 3, red/black preconditioning).  A site of
// parity p = (x+y+z+t) mod 2 with lexicographic index s has the compact
// index h = s / 2 in the half-lattice array of its parity (x extent even).
// Half-lattice fields are [rhs][colour][Vhs][spin]: the four spins of one
// colour at one site are adjacent, so a lane reads them with one 16-byte
// (FP16), two (FP32) or four (FP64) loads and projects them at once.  Links
// are [parity][4][NR][Vhs].  The hopping term between the sublattices,
// H_p(v) at sites of parity p from v on the other one, is the sum over mu of
// (1 - gamma_mu) U_mu(x) v(x+mu) + (1 + gamma_mu) U_mu(x-mu)^dag v(x-mu);
// D_{p,1-p} = -H_p / 2.
struct EoGeom {
  int L[4];
  int hx;        // compact sites per x line (L0 / 2)
  long Vh, Vhs;  // sites per parity, compact array stride
  long Vsf;      // site stride of full-lattice fields
};


// Work order of the hop kernels.  A tile is 256 consecutive compact sites of
// a slab of zb z-slices at one t (x fastest, then y, then z inside the
// slab); tiles are numbered slab chunk fastest, then t, then z-slab, and XCD
// k takes the k-th contiguous range.  The t-neighbours of a tile are then a
// few tiles away in the XCD's sequence.  The rhs tiles are swept in groups of
// grp: an XCD runs its whole range for one group before the next, with the
// group's rhs tiles of one site tile back to back.  One group holding every
// rhs tile reads the links once; smaller groups read them once per group but
// bring the t-neighbours closer in the sequence (8 rhs tiles of 256 sites and
// three FP16 rhs each already touch about 1 MB, against a 4 MB L2 per XCD).
struct EoTiles {
  int zb;     // z-slices per slab (divides L2)
  int nch;    // chunks of 256 sites per slab and t
  int ntile;  // tiles
  int tpx;    // tiles per XCD
  int grp;    // rhs tiles per group
  int nt;     // FP16 diagonal input and output with the non-temporal hint
};

static EoTiles make_eo_tiles(const EoGeom &e, int zb, int grp, int nt = 0) {
  EoTiles t;
  t.zb = zb;
  const long q = (long)e.hx * e.L[1] * zb;
  t.nch = (int)((q + 255) / 256);
  t.ntile = t.nch * e.L[3] * (e.L[2] / zb);
  t.tpx = (t.ntile + NXCD - 1) / NXCD;
  t.grp = grp < 1 ? 1 : grp;
  t.nt = nt;
  return t;
}

// The compact site of one thread of a hop kernel: tile and first rhs from
// the block (groups of rhs tiles, XCD ranges), coordinates from the lane.
struct EoSite {
  int tile, r0;    // tile index, first rhs of the thread
  int x[4], h, xh; // coordinates, compact index, compact x
  bool valid_tile, valid;
};

__device__ __forceinline__ EoSite eo_site(const EoGeom &g, const EoTiles &tl, int par, int nrhs, int RT) {
  EoSite s;
  const int nrt = (nrhs + RT - 1) / RT;
  const int j = (int)(blockIdx.x / NXCD);
  const int span = tl.tpx * tl.grp;           // blocks of one full group on an XCD
  const int g0 = (j / span) * tl.grp;         // first rhs tile of this block's group
  const int gc = min(tl.grp, nrt - g0);       // rhs tiles in the group (the last may be short)
  const int rem = j - (g0 / tl.grp) * span;
  s.tile = (int)(blockIdx.x % NXCD) * tl.tpx + rem / gc;
  s.r0 = (g0 + rem % gc) * RT;
  s.valid_tile = s.tile < tl.ntile;
  s.valid = false;
  s.x[0] = s.x[1] = s.x[2] = s.x[3] = 0;
  s.h = s.xh = 0;
  if (s.valid_tile) {
    const int P = g.hx * g.L[1];
    const int u = s.tile / tl.nch;
    const int q = (s.tile - u * tl.nch) * 256 + (int)threadIdx.x;
    const int tt = u % g.L[3];
    const int zi = q / P, hp = q - zi * P;
    s.valid = zi < tl.zb;
    s.x[1] = hp / g.hx;
    s.xh = hp - s.x[1] * g.hx;
    s.x[2] = (u / g.L[3]) * tl.zb + zi;
    s.x[3] = tt;
    s.x[0] = 2 * s.xh + ((par + s.x[1] + s.x[2] + s.x[3]) & 1);
    s.h = hp + P * (s.x[2] + g.L[2] * tt);
  }
  return s;
}

// compact indices of the forward and backward neighbours in direction MU
template <int MU>
__device__ __forceinline__ void eo_neighbours(const EoGeom &g, const EoSite &s, int &hf, int &hb) {
  if (MU == 0) {
    const int xf = s.x[0] == g.L[0] - 1 ? 0 : s.x[0] + 1;
    const int xb = s.x[0] == 0 ? g.L[0] - 1 : s.x[0] - 1;
    hf = s.h - s.xh + (xf >> 1);
    hb = s.h - s.xh + (xb >> 1);
  } else {
    const int hs = MU == 1 ? g.hx : (MU == 2 ? g.hx * g.L[1] : g.hx * g.L[1] * g.L[2]);
    hf = s.x[MU] == g.L[MU] - 1 ? s.h - (g.L[MU] - 1) * hs : s.h + hs;
    hb = s.x[MU] == 0 ? s.h + (g.L[MU] - 1) * hs : s.h - hs;
  }
}

// out = a in_diag + b acc per rhs of the thread (see k_hop_eo for ADD),
// with the reduction terms of RED accumulated into rs
template <class TD, class TH, class TO, int RT, int RED, int ADD, class R>
__device__ __forceinline__ void eo_store(const EoGeom &g, const EoTiles &tl, const EoSite &st, int nrhs,
                                         const TD *__restrict__ in_diag, const TH *__restrict__ in_hop,
                                         TO *__restrict__ out, double ad, R a, R b, cx<R> (&acc)[RT][12],
                                         double (&rs)[RT][3], const __half2 *__restrict__ ebase = nullptr) {
  const int Vs = (int)g.Vhs;
  // a thread's reduction terms summed in the arithmetic's precision (12
  // products per rhs), then added to the FP64 block sums
  using A = typename std::conditional<sizeof(R) == 8, double, float>::type;
#pragma unroll
  for (int t = 0; t < RT; t++) {
    if (st.r0 + t >= nrhs) continue;
    A loc[3] = {A(0), A(0), A(0)};
#pragma unroll
    for (int c = 0; c < 3; c++) {
      const size_t i = ((size_t)(st.r0 + t) * 3 + c) * Vs * 4 + (unsigned)st.h * 4;
      cx<R> dv[4] = {czero<R>(), czero<R>(), czero<R>(), czero<R>()};
      if (ad != 0.0) {
        if (tl.nt) ld4_nt(in_diag + i, dv);
        else ld4(in_diag + i, dv);
      }
      cx<R> o[4];
#pragma unroll
      for (int sp = 0; sp < 4; sp++)
        o[sp] = {a * dv[sp].re + b * acc[t][sp * 3 + c].re, a * dv[sp].im + b * acc[t][sp * 3 + c].im};
      if constexpr (ADD) {
        // the pair (2h, 2h + 1) of full-lattice sites: this site and its
        // partner of the other parity
        cx<R> hv[4];
        ld4(in_hop + i, hv);
        const int own = st.x[0] & 1;
#pragma unroll
        for (int sp = 0; sp < 4; sp++) {
          const size_t fi = ((size_t)(st.r0 + t) * 12 + sp * 3 + c) * g.Vsf + 2 * (size_t)(unsigned)st.h;
          if constexpr (ADD == 2) set_pair_base(out + fi, ebase + fi, own ? hv[sp] : o[sp], own ? o[sp] : hv[sp]);
          else add_pair(out + fi, own ? hv[sp] : o[sp], own ? o[sp] : hv[sp]);
        }
      } else if (tl.nt) {
        st4_nt(out + i, o);
      } else {
        st4(out + i, o);
      }
      if (RED) {
#pragma unroll
        for (int sp = 0; sp < 4; sp++) {
          const cx<R> os = as_stored(out, o[sp]);
          loc[0] += (A)os.re * (A)dv[sp].re + (A)os.im * (A)dv[sp].im;
          loc[1] += (A)os.re * (A)dv[sp].im - (A)os.im * (A)dv[sp].re;
          loc[2] += (A)os.re * (A)os.re + (A)os.im * (A)os.im;
        }
      }
    }
    if (RED) {
      rs[t][0] += (double)loc[0];
      rs[t][1] += (double)loc[1];
      rs[t][2] += (double)loc[2];
    }
  }
}

// block sums of the RED terms -> red[(rhs * ntile + tile) * 3 + k]; every
// thread of the block calls it
template <int RT>
__device__ __forceinline__ void eo_reduce(const EoTiles &tl, const EoSite &st, int nrhs, double (&rs)[RT][3],
                                          double *__restrict__ red) {
  __shared__ double sh[RT][3][4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int t = 0; t < RT; t++)
#pragma unroll
    for (int k = 0; k < 3; k++) {
      double v = rs[t][k];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
      if (lane == 0) sh[t][k][wv] = v;
    }
  __syncthreads();
  if (st.valid_tile && threadIdx.x < RT * 3) {
    const int t = threadIdx.x / 3, k = threadIdx.x % 3;
    if (st.r0 + t < nrhs)
      red[((size_t)(st.r0 + t) * tl.ntile + st.tile) * 3 + k] = sh[t][k][0] + sh[t][k][1] + sh[t][k][2] + sh[t][k][3];
  }
}

// out = a in_diag + b H_par(in_hop) at the compact sites of parity par, for
// RT right-hand sides per thread (sharing every link load), with FP32 or
// FP64 arithmetic; with RED, also <out, in_diag> and |out|^2 per tile and
// rhs into red (as stored).  With ADD, out is instead a full-lattice field
// [rhs][12][Vsf] that receives the result at the site of parity par and
// in_hop's value at the other site of the same x pair (same compact index):
// the last step of the red/black smoother, e += (d_e, d_o) (ADD = 1), or
// out = ebase + (d_e, d_o) with ebase an FP16 full-lattice field (ADD = 2),
// without a separate pass.  Site indices are 32-bit (a parity holds fewer
// than 2^29 sites).
template <class TL, class TD, class TH, class TO, int RT, int RED, int NR, int ADD = 0>
__global__ void __launch_bounds__(256) k_hop_eo(const TL *__restrict__ Ue, const TD *__restrict__ in_diag,
                                               const TH *__restrict__ in_hop, TO *__restrict__ out, EoGeom g, int par,
                                               double ad, double bd, int nrhs, EoTiles tl, double *__restrict__ red,
                                               float one, const __half2 *__restrict__ ebase) {
  using R = typename store_traits<TO>::real;
  const EoSite st = eo_site(g, tl, par, nrhs, RT);
  const int r0 = st.r0;
  double rs[RT][3];
#pragma unroll
  for (int t = 0; t < RT; t++) rs[t][0] = rs[t][1] = rs[t][2] = 0.0;
  if (st.valid) {
    const int Vs = (int)g.Vhs;
    const TL *Uf = Ue + (size_t)par * 4 * NR * Vs;        // links at sites of parity par
    const TL *Ub = Ue + (size_t)(1 - par) * 4 * NR * Vs;  // ... of the other parity
    cx<R> acc[RT][12];
#pragma unroll
    for (int t = 0; t < RT; t++)
#pragma unroll
      for (int c = 0; c < 12; c++) acc[t][c] = czero<R>();
    auto load_link = [&](const TL *Up, int mu, int site, cx<R> u[9]) {
#pragma unroll
      for (int e = 0; e < NR; e++) {
        auto v = ldc(Up + (size_t)(mu * NR + e) * Vs + (unsigned)site);
        u[e] = {(R)v.re, (R)v.im};
      }
      if (NR == 6) su3_third_row(u);
    };
    // projected half spinor of the neighbour, colour by colour
    auto half = [&](int r, int site, auto proj, cx<R> hh[6]) {
#pragma unroll
      for (int c = 0; c < 3; c++) {
        cx<R> p4[4];
        ld4(in_hop + ((size_t)r * 3 + c) * Vs * 4 + (unsigned)site * 4, p4);
        proj(p4, hh[c], hh[3 + c]);
      }
    };
#define EO_DIR(MU)                                                                      \
    {                                                                                   \
      int hf, hb;                                                                       \
      eo_neighbours<MU>(g, st, hf, hb);                                                 \
      cx<R> u[9], hh[6], gg[6];                                                         \
      load_link(Uf, MU, st.h, u);                                                       \
      _Pragma("unroll") for (int t = 0; t < RT; t++) {                                  \
        if (r0 + t < nrhs) {                                                            \
          half(r0 + t, hf, proj_pair<MU, 1, R>, hh);                                    \
          su3_mul<0>(u, hh, gg);                                                        \
          reconstruct<MU, 1>(gg, acc[t]);                                               \
        }                                                                               \
      }                                                                                 \
      load_link(Ub, MU, hb, u);                                                         \
      _Pragma("unroll") for (int t = 0; t < RT; t++) {                                  \
        if (r0 + t < nrhs) {                                                            \
          half(r0 + t, hb, proj_pair<MU, -1, R>, hh);                                   \
          su3_mul<1>(u, hh, gg);                                                        \
          reconstruct<MU, -1>(gg, acc[t]);                                              \
        }                                                                               \
      }                                                                                 \
    }
    EO_DIR(0)
    EO_DIR(1)
    EO_DIR(2)
    EO_DIR(3)
#undef EO_DIR
    eo_store<TD, TH, TO, RT, RED, ADD, R>(g, tl, st, nrhs, in_diag, in_hop, out, ad, (R)ad, (R)bd, acc, rs, ebase);
  }
  if (RED) eo_reduce<RT>(tl, st, nrhs, rs, red);
}

// ---- packed FP16 form
// The all-FP16 hop of the smoother's MR steps computes the spin projection,
// the SU(3) products and the sum and difference of the forward and backward
// terms of each direction in packed half precision: two FP16 values per lane
// and instruction, with the complex broadcasts, swaps and signs folded into
// the operands' modifiers (a complex multiply-add is two packed FMAs).  The
// eight directions are accumulated in FP32 (the FP16 -> FP32 conversion
// folded into the FMA through `one`, as above), and the output is formed and
// rounded as in k_hop_eo.  The FP16 products round at 2^-11 relative to the
// link and spinor magnitudes, the size of the FP16 storage rounding of the
// same fields.
template <int RT, int RED, int NR, int ADD = 0>
__global__ void __launch_bounds__(256) k_hop_eo_pk(const __half2 *__restrict__ Ue, const __half2 *__restrict__ in_diag,
                                                  const __half2 *__restrict__ in_hop, __half2 *__restrict__ out,
                                                  EoGeom g, int par, double ad, double bd, int nrhs, EoTiles tl,
                                                  double *__restrict__ red, float one,
                                                  const __half2 *__restrict__ ebase) {
  const EoSite st = eo_site(g, tl, par, nrhs, RT);
  const int r0 = st.r0;
  double rs[RT][3];
#pragma unroll
  for (int t = 0; t < RT; t++) rs[t][0] = rs[t][1] = rs[t][2] = 0.0;
  if (st.valid) {
    const int Vs = (int)g.Vhs;
    const __half2 *Uf = Ue + (size_t)par * 4 * NR * Vs;
    const __half2 *Ub = Ue + (size_t)(1 - par) * 4 * NR * Vs;
    cx<float> acc[RT][12];
#pragma unroll
    for (int t = 0; t < RT; t++)
#pragma unroll
      for (int c = 0; c < 12; c++) acc[t][c] = {0.f, 0.f};
#define PK_DIR(MU)                                                                                  \
    {                                                                                               \
      int hf, hb;                                                                                   \
      eo_neighbours<MU>(g, st, hf, hb);                                                             \
      h2 uf[9], ub[9];                                                                              \
      pk_link<NR>(Uf, MU, (unsigned)st.h, Vs, uf);                                                  \
      pk_link<NR>(Ub, MU, (unsigned)hb, Vs, ub);                                                    \
      _Pragma("unroll") for (int t = 0; t < RT; t++) {                                              \
        if (r0 + t < nrhs) {                                                                        \
          const __half2 *in_r = in_hop + (size_t)(r0 + t) * 3 * Vs * 4;                             \
          h2 hh[6], gf[6], gb[6];                                                                   \
          _Pragma("unroll") for (int c = 0; c < 3; c++)                                             \
            pk_proj<MU, 1>(in_r + (size_t)c * Vs * 4 + (unsigned)hf * 4, hh[c], hh[3 + c]);         \
          _Pragma("unroll") for (int sp = 0; sp < 2; sp++)                                          \
          _Pragma("unroll") for (int a = 0; a < 3; a++) {                                           \
            h2 v = pk_cmul(uf[3 * a], hh[3 * sp]);                                                  \
            v = pk_cfma(uf[3 * a + 1], hh[3 * sp + 1], v);                                          \
            gf[3 * sp + a] = pk_cfma(uf[3 * a + 2], hh[3 * sp + 2], v);                             \
          }                                                                                         \
          _Pragma("unroll") for (int c = 0; c < 3; c++)                                             \
            pk_proj<MU, -1>(in_r + (size_t)c * Vs * 4 + (unsigned)hb * 4, hh[c], hh[3 + c]);        \
          _Pragma("unroll") for (int sp = 0; sp < 2; sp++)                                          \
          _Pragma("unroll") for (int a = 0; a < 3; a++) {                                           \
            h2 v = pk_cfmac(ub[a], hh[3 * sp], (h2){0, 0});                                         \
            v = pk_cfmac(ub[3 + a], hh[3 * sp + 1], v);                                             \
            gb[3 * sp + a] = pk_cfmac(ub[6 + a], hh[3 * sp + 2], v);                                \
          }                                                                                         \
          pk_recon<MU>(gf, gb, acc[t], one);                                                        \
        }                                                                                           \
      }                                                                                             \
    }
    PK_DIR(0)
    PK_DIR(1)
    PK_DIR(2)
    PK_DIR(3)
#undef PK_DIR
    eo_store<__half2, __half2, __half2, RT, RED, ADD, float>(g, tl, st, nrhs, in_diag, in_hop, out, ad, (float)ad,
                                                             (float)bd, acc, rs, ebase);
  }
  if (RED) eo_reduce<RT>(tl, st, nrhs, rs, red);
}

static EoGeom make_eo(const Geom &g) {
  EoGeom e;
  for (int i = 0; i < 4; i++) e.L[i] = g.L[i];
  e.hx = g.L[0] / 2;
  e.Vh = g.V / 2;
  e.Vhs = fine_stride(e.Vh);
  e.Vsf = g.Vs;
  return e;
}

long eo_stride(const Geom &g) { return fine_stride(g.V / 2); }

// slab depths the autotuner tries (those dividing L2), the first the default
static int eo_zb_candidates(const Geom &g, int zb[6]) {
  const int pref[6] = {4, 8, 2, 1, 16, g.L[2]};
  int n = 0;
  for (int i = 0; i < 6; i++) {
    if (pref[i] < 1 || g.L[2] % pref[i]) continue;
    bool dup = false;
    for (int k = 0; k < n; k++) dup |= zb[k] == pref[i];
    if (!dup) zb[n++] = pref[i];
  }
  return n;
}

// (slab depth, rhs tiles per group, non-temporal hint) triples the
// autotuner tries for nrt rhs tiles: every slab depth with one group, then
// slab depths 4 and 2 with groups of 2 to 5 rhs tiles, then slab depths 4, 2
// and 8 with one group and the hint (FP16 only); the first is the default
static int eo_tile_candidates(const Geom &g, int nrt, bool h16, int zb[20], int grp[20], int nt[20]) {
  int z[6];
  const int nz = eo_zb_candidates(g, z);
  int n = 0;
  for (int i = 0; i < nz; i++) {
    zb[n] = z[i];
    grp[n] = nrt;
    nt[n++] = 0;
  }
  const int zg[2] = {4, 2}, gs[4] = {4, 3, 2, 5};
  for (int a = 0; a < 2; a++) {
    if (zg[a] > g.L[2] || g.L[2] % zg[a]) continue;
    for (int b = 0; b < 4; b++) {
      if (gs[b] >= nrt) continue;
      zb[n] = zg[a];
      grp[n] = gs[b];
      nt[n++] = 0;
    }
  }
  const int zn[3] = {4, 2, 8};
  for (int a = 0; a < 3 && h16; a++) {
    if (zn[a] > g.L[2] || g.L[2] % zn[a]) continue;
    zb[n] = zn[a];
    grp[n] = nrt;
    nt[n++] = 1;
  }
  return n;
}

long eo_red_tiles(const Geom &g) {
  EoGeom e = make_eo(g);
  int zb[6];
  const int n = eo_zb_candidates(g, zb);
  long m = 0;
  for (int i = 0; i < n; i++) {
    const long t = make_eo_tiles(e, zb[i], 1).ntile;
    m = t > m ? t : m;
  }
  return m;
}

template <class TL, class TD, class TH, class TO, int RT, int NR, int ADD = 0>
static int launch_hop_eo(const Geom &g, const void *Ue, int par, double a, double b, const void *in_diag,
                         const void *in_hop, void *out, int nrhs, double *red, double *red_out, int red_stride,
                         hipStream_t st, const void *ebase = nullptr) {
  EoGeom e = make_eo(g);
  const int nrt = (nrhs + RT - 1) / RT;
  int zb[20], grp[20], nt[20];
  const int ncand = eo_tile_candidates(g, nrt, std::is_same<TO, __half2>::value, zb, grp, nt);
  // the all-FP16 form runs the packed-arithmetic kernel (also the fused
  // full-lattice write from an FP16 base, ADD 2, with FP16 output)
  constexpr bool pk = std::is_same<TL, __half2>::value && std::is_same<TD, __half2>::value &&
                      std::is_same<TH, __half2>::value && std::is_same<TO, __half2>::value && ADD != 1;
  auto run = [&](int cand) -> int {
    const EoTiles tl = make_eo_tiles(e, zb[cand], grp[cand], nt[cand]);
    const dim3 grid((unsigned)((long)NXCD * tl.tpx * nrt));
    if constexpr (pk) {
      if (red)
        hipLaunchKernelGGL((k_hop_eo_pk<RT, 1, NR>), grid, dim3(256), 0, st, (const __half2 *)Ue,
                           (const __half2 *)in_diag, (const __half2 *)in_hop, (__half2 *)out, e, par, a, b, nrhs, tl,
                           red, 1.0f, (const __half2 *)nullptr);
      else
        hipLaunchKernelGGL((k_hop_eo_pk<RT, 0, NR, ADD>), grid, dim3(256), 0, st, (const __half2 *)Ue,
                           (const __half2 *)in_diag, (const __half2 *)in_hop, (__half2 *)out, e, par, a, b, nrhs, tl,
                           (double *)nullptr, 1.0f, (const __half2 *)ebase);
    } else if (red) {
      hipLaunchKernelGGL((k_hop_eo<TL, TD, TH, TO, RT, 1, NR>), grid, dim3(256), 0, st, (const TL *)Ue,
                         (const TD *)in_diag, (const TH *)in_hop, (TO *)out, e, par, a, b, nrhs, tl, red, 1.0f,
                         (const __half2 *)nullptr);
    } else {
      hipLaunchKernelGGL((k_hop_eo<TL, TD, TH, TO, RT, 0, NR, ADD>), grid, dim3(256), 0, st, (const TL *)Ue,
                         (const TD *)in_diag, (const TH *)in_hop, (TO *)out, e, par, a, b, nrhs, tl,
                         (double *)nullptr, 1.0f, (const __half2 *)ebase);
    }
    if (red)
      hipLaunchKernelGGL(k_dslash_red_finalize, dim3(nrhs), dim3(256), 0, st, red, (long)tl.ntile, red_out,
                         red_stride);
    WMG_HIP(hipGetLastError());
    return 0;
  };
  char key[256];
  std::snprintf(key, sizeof(key), "hop_eo/l%zu-d%zu-h%zu-o%zu-nr%d-red%d-diag%d-add%d/%dx%dx%dx%d/rhs%d",
                sizeof(TL), sizeof(TD), sizeof(TH), sizeof(TO), NR, red ? 1 : 0, a != 0.0 ? 1 : 0, ADD, g.L[0],
                g.L[1], g.L[2], g.L[3], nrhs);
  int choice = 0;
  // candidates with ADD accumulate into out: not pure, so no search (slab
  // depth 4, or the first that divides L2)
  return ADD ? run(0) : tune_choice(key, ncand, run, st, &choice);
}

int hop_eo(const Geom &g, int lprec, const void *Ue, int par, double a, double b, int pdiag, const void *in_diag,
           int phop, const void *in_hop, int pout, void *out, int nrhs, double *red, double *red_out, int red_stride,
           hipStream_t st) {
  const bool c12 = (lprec & LK12) != 0;
  const int lp = lprec & ~LK12;
  if (g.L[0] % 2 || g.V / 2 >= (1L << 29)) return set_error(-1, "hop_eo: lattice not supported");
#define HOP(TL, TD, TH, TO, RT)                                                                                    \
  return c12 ? launch_hop_eo<TL, TD, TH, TO, RT, 6>(g, Ue, par, a, b, in_diag, in_hop, out, nrhs, red, red_out,    \
                                                   red_stride, st)                                                \
             : launch_hop_eo<TL, TD, TH, TO, RT, 9>(g, Ue, par, a, b, in_diag, in_hop, out, nrhs, red, red_out,    \
                                                   red_stride, st)
  if (lp == P64 && pdiag == P64 && phop == P64 && pout == P64) HOP(double2, double2, double2, double2, 1);
  if (lp == P16 && pdiag == P16 && phop == P16 && pout == P16) HOP(__half2, __half2, __half2, __half2, 4);
  if (lp == P16 && pdiag == P16 && phop == P32 && pout == P32) HOP(__half2, __half2, float2, float2, 2);
#undef HOP
  return set_error(-1, "hop_eo: unsupported precisions link %d diag %d hop %d out %d", lp, pdiag, phop, pout);
}

int hop_eo_add(const Geom &g, int lprec, const void *Ue, double a, double b, int pdiag, const void *in_diag,
               int phop, const void *de, void *full, int nrhs, hipStream_t st, const void *ebase, int pfull) {
  const bool c12 = (lprec & LK12) != 0;
  const int lp = lprec & ~LK12;
  if (g.L[0] % 2 || g.V / 2 >= (1L << 29)) return set_error(-1, "hop_eo_add: lattice not supported");
  if (pfull == P16) {
    if (!(lp == P16 && pdiag == P16 && phop == P16 && ebase))
      return set_error(-1, "hop_eo_add: FP16 full-lattice output only from an FP16 base with FP16 fields");
    return c12 ? launch_hop_eo<__half2, __half2, __half2, __half2, 4, 6, 2>(g, Ue, 1, a, b, in_diag, de, full, nrhs,
                                                                            nullptr, nullptr, 0, st, ebase)
               : launch_hop_eo<__half2, __half2, __half2, __half2, 4, 9, 2>(g, Ue, 1, a, b, in_diag, de, full, nrhs,
                                                                            nullptr, nullptr, 0, st, ebase);
  }
  if (pfull != P32 && pfull != P64) return set_error(-1, "hop_eo_add: output precision %d", pfull);
#define HOPA(TL, TD, TH, TO, RT)                                                                                  \
  return c12 ? launch_hop_eo<TL, TD, TH, TO, RT, 6, 1>(g, Ue, 1, a, b, in_diag, de, full, nrhs, nullptr, nullptr, 0, \
                                                      st)                                                          \
             : launch_hop_eo<TL, TD, TH, TO, RT, 9, 1>(g, Ue, 1, a, b, in_diag, de, full, nrhs, nullptr, nullptr, 0, st)
  if (lp == P64 && pdiag == P64 && phop == P64) HOPA(double2, double2, double2, double2, 1);
  if (lp == P16 && pdiag == P16 && phop == P32) HOPA(__half2, __half2, float2, float2, 2);
  if (lp == P16 && pdiag == P16 && phop == P16 && ebase)
    return c12 ? launch_hop_eo<__half2, __half2, __half2, float2, 2, 6, 2>(g, Ue, 1, a, b, in_diag, de, full, nrhs,
                                                                          nullptr, nullptr, 0, st, ebase)
               : launch_hop_eo<__half2, __half2, __half2, float2, 2, 9, 2>(g, Ue, 1, a, b, in_diag, de, full, nrhs,
                                                                          nullptr, nullptr, 0, st, ebase);
  if (lp == P16 && pdiag == P16 && phop == P16) HOPA(__half2, __half2, __half2, float2, 2);
#undef HOPA
  return set_error(-1, "hop_eo_add: unsupported precisions link %d diag %d field %d", lp, pdiag, phop);
}

// full lexicographic SoA [rhs][12][Vs] <-> half-lattice [rhs][colour][Vhs][spin]
template <class TF, class TE>
__global__ void k_eo_pack(const TF *__restrict__ full, TE *__restrict__ ev, TE *__restrict__ od, EoGeom g, long Vs) {
  using R = typename store_traits<TE>::real;
  long s = blockIdx.x * 256L + threadIdx.x;
  int r = blockIdx.y;
  if (s >= 2 * g.Vh) return;
  int x[4];
  site_coords(g.L, s, x);
  TE *dst = ((x[0] + x[1] + x[2] + x[3]) & 1) ? od : ev;
  const long hh = s >> 1;
#pragma unroll
  for (int c = 0; c < 3; c++) {
    cx<R> o[4];
#pragma unroll
    for (int sp = 0; sp < 4; sp++) {
      auto v = ldc(full + ((size_t)r * 12 + sp * 3 + c) * Vs + s);
      o[sp] = {(R)v.re, (R)v.im};
    }
    st4(dst + (((size_t)r * 3 + c) * g.Vhs + hh) * 4, o);
  }
}
// full += (ev, od) (either half may be null: no contribution)
template <class TF, class TE>
__global__ void k_eo_unpack_add(TF *__restrict__ full, const TE *__restrict__ ev, const TE *__restrict__ od, EoGeom g,
                                long Vs) {
  using R = typename store_traits<TE>::real;
  long s = blockIdx.x * 256L + threadIdx.x;
  int r = blockIdx.y;
  if (s >= 2 * g.Vh) return;
  int x[4];
  site_coords(g.L, s, x);
  const TE *src = ((x[0] + x[1] + x[2] + x[3]) & 1) ? od : ev;
  if (!src) return;
  const long hh = s >> 1;
#pragma unroll
  for (int c = 0; c < 3; c++) {
    cx<R> v[4];
    ld4(src + (((size_t)r * 3 + c) * g.Vhs + hh) * 4, v);
#pragma unroll
    for (int sp = 0; sp < 4; sp++) {
      const size_t i = ((size_t)r * 12 + sp * 3 + c) * Vs + s;
      auto f = ldc(full + i);
      stc(full + i, decltype(f){f.re + v[sp].re, f.im + v[sp].im});
    }
  }
}

int eo_pack(const Geom &g, int pfull, const void *full, int phalf, void *ev, void *od, int nrhs, hipStream_t st) {
  EoGeom e = make_eo(g);
  dim3 grid((unsigned)((g.V + 255) / 256), nrhs);
  if (pfull == P16 && phalf == P16)
    hipLaunchKernelGGL((k_eo_pack<__half2, __half2>), grid, dim3(256), 0, st, (const __half2 *)full, (__half2 *)ev,
                       (__half2 *)od, e, g.Vs);
  else if (pfull == P32 && phalf == P32)
    hipLaunchKernelGGL((k_eo_pack<float2, float2>), grid, dim3(256), 0, st, (const float2 *)full, (float2 *)ev,
                       (float2 *)od, e, g.Vs);
  else if (pfull == P64 && phalf == P64)
    hipLaunchKernelGGL((k_eo_pack<double2, double2>), grid, dim3(256), 0, st, (const double2 *)full, (double2 *)ev,
                       (double2 *)od, e, g.Vs);
  else return set_error(-1, "eo_pack: precisions %d -> %d", pfull, phalf);
  WMG_HIP(hipGetLastError());
  return 0;
}

int eo_unpack_add(const Geom &g, int pfull, void *full, int phalf, const void *ev, const void *od, int nrhs,
                  hipStream_t st) {
  EoGeom e = make_eo(g);
  dim3 grid((unsigned)((g.V + 255) / 256), nrhs);
  if (pfull == P32 && phalf == P32)
    hipLaunchKernelGGL((k_eo_unpack_add<float2, float2>), grid, dim3(256), 0, st, (float2 *)full, (const float2 *)ev,
                       (const float2 *)od, e, g.Vs);
  else if (pfull == P64 && phalf == P64)
    hipLaunchKernelGGL((k_eo_unpack_add<double2, double2>), grid, dim3(256), 0, st, (double2 *)full,
                       (const double2 *)ev, (const double2 *)od, e, g.Vs);
  else return set_error(-1, "eo_unpack_add: precisions %d <- %d", pfull, phalf);
  WMG_HIP(hipGetLastError());
  return 0;
}

// links [4][9][Vs] (FP64, whole, lexicographic SoA) -> [parity][4][NR][Vhs]
template <class TL, int NR>
__global__ void k_links_to_eo(const double2 *__restrict__ U, TL *__restrict__ Ue, EoGeom g, long Vs) {
  long s = blockIdx.x * 256L + threadIdx.x;
  if (s >= 2 * g.Vh) return;
  int x[4];
  site_coords(g.L, s, x);
  const int par = (x[0] + x[1] + x[2] + x[3]) & 1;
  const long hh = s >> 1;
  for (int mu = 0; mu < 4; mu++)
    for (int e = 0; e < NR; e++) {
      double2 v = U[(size_t)(mu * 9 + e) * Vs + s];
      TL *d = Ue + ((size_t)(par * 4 + mu) * NR + e) * g.Vhs + hh;
      if constexpr (sizeof(TL) == 16) *d = v;
      else if constexpr (sizeof(TL) == 8) *d = make_float2((float)v.x, (float)v.y);
      else *d = __floats2half2_rn((float)v.x, (float)v.y);
    }
}

int links_to_eo(const Geom &g, const void *U64soa, int lprec, void *Ue, hipStream_t st) {
  EoGeom e = make_eo(g);
  dim3 grid((unsigned)((g.V + 255) / 256));
  const bool c12 = (lprec & LK12) != 0;
  const int lp = lprec & ~LK12;
#define L2E(TL)                                                                                                     \
  do {                                                                                                            \
    if (c12) hipLaunchKernelGGL((k_links_to_eo<TL, 6>), grid, dim3(256), 0, st, (const double2 *)U64soa, (TL *)Ue, e, g.Vs); \
    else hipLaunchKernelGGL((k_links_to_eo<TL, 9>), grid, dim3(256), 0, st, (const double2 *)U64soa, (TL *)Ue, e, g.Vs);     \
  } while (0)
  if (lp == P64) L2E(double2);
  else if (lp == P32) L2E(float2);
  else L2E(__half2);
#undef L2E
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
template <class TL, int NR>
__global__ void k_links_to_soa(const double2 *__restrict__ Uc, TL *__restrict__ Us, long V, long Vs) {
  long s = blockIdx.x * 256L + threadIdx.x;
  if (s >= V) return;
  for (int mu = 0; mu < 4; mu++)
    for (int e = 0; e < NR; e++) {
      double2 v = Uc[(s * 4 + mu) * 9 + e];
      TL *d = Us + (size_t)(mu * NR + e) * Vs + s;
      if constexpr (sizeof(TL) == 16) *d = v;
      else if constexpr (sizeof(TL) == 8) *d = make_float2((float)v.x, (float)v.y);
      else *d = __floats2half2_rn((float)v.x, (float)v.y);
    }
}

int links_to_soa(const Geom &g, const double *Ucanon, int lprec, void *Usoa, hipStream_t st) {
  dim3 grid((unsigned)((g.V + 255) / 256));
  const bool c12 = (lprec & LK12) != 0;
  const int lp = lprec & ~LK12;
#define L2S(TL)                                                                                                  \
  do {                                                                                                         \
    if (c12) hipLaunchKernelGGL((k_links_to_soa<TL, 6>), grid, dim3(256), 0, st, (const double2 *)Ucanon, (TL *)Usoa, g.V, g.Vs); \
    else hipLaunchKernelGGL((k_links_to_soa<TL, 9>), grid, dim3(256), 0, st, (const double2 *)Ucanon, (TL *)Usoa, g.V, g.Vs);     \
  } while (0)
  if (lp == P64) L2S(double2);
  else if (lp == P32) L2S(float2);
  else L2S(__half2);
#undef L2S
  WMG_HIP(hipGetLastError());
  return 0;
}

// Largest |row2 - conj(row0 x row1)| of the canonical FP64 links in each
// workgroup of 256 sites -> part[block]: zero (to rounding) exactly when
// the 12-real format reproduces the field.
__global__ void __launch_bounds__(256) k_su3_recon_err(const double2 *__restrict__ Uc, long V, double *__restrict__ part) {
  long s = blockIdx.x * 256L + threadIdx.x;
  double e = 0;
  if (s < V)
    for (int mu = 0; mu < 4; mu++) {
      cx<double> u[9];
      for (int k = 0; k < 9; k++) u[k] = ldc(Uc + (s * 4 + mu) * 9 + k);
      cx<double> w[9];
      for (int k = 0; k < 6; k++) w[k] = u[k];
      su3_third_row(w);
      for (int k = 6; k < 9; k++) e = fmax(e, fmax(fabs(w[k].re - u[k].re), fabs(w[k].im - u[k].im)));
    }
  __shared__ double sh[4];
  for (int o = 32; o > 0; o >>= 1) e = fmax(e, __shfl_down(e, o, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = e;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

long su3_recon_blocks(const Geom &g) { return (g.V + 255) / 256; }

int su3_recon_err(const Geom &g, const double *Ucanon, double *part, hipStream_t st) {
  hipLaunchKernelGGL(k_su3_recon_err, dim3((unsigned)su3_recon_blocks(g)), dim3(256), 0, st, (const double2 *)Ucanon,
                     g.V, part);
  WMG_HIP(hipGetLastError());
  return 0;
}

// canonical [rhs][V][12] <-> SoA [rhs][12][Vs], 256 sites per workgroup
// through LDS so that both sides are read and written in contiguous runs
// (rows padded to 257 elements against bank conflicts)
__global__ void __launch_bounds__(256) k_spinor_to_soa(const double2 *__restrict__ c, double2 *__restrict__ s, long V,
                                                      long Vs) {
  __shared__ double2 t[12 * 257];
  const long i0 = blockIdx.x * 256L;
  const int r = blockIdx.y;
  const int nv = (int)(V - i0 < 256 ? V - i0 : 256);
  const double2 *src = c + ((size_t)r * V + i0) * 12;
  for (int q = threadIdx.x; q < nv * 12; q += 256) t[(q % 12) * 257 + q / 12] = src[q];
  __syncthreads();
  if ((int)threadIdx.x < nv)
#pragma unroll
    for (int k = 0; k < 12; k++) s[((size_t)r * 12 + k) * Vs + i0 + threadIdx.x] = t[k * 257 + threadIdx.x];
}
__global__ void __launch_bounds__(256) k_spinor_from_soa(const double2 *__restrict__ s, double2 *__restrict__ c,
                                                        long V, long Vs) {
  __shared__ double2 t[12 * 257];
  const long i0 = blockIdx.x * 256L;
  const int r = blockIdx.y;
  const int nv = (int)(V - i0 < 256 ? V - i0 : 256);
  if ((int)threadIdx.x < nv)
#pragma unroll
    for (int k = 0; k < 12; k++) t[k * 257 + threadIdx.x] = s[((size_t)r * 12 + k) * Vs + i0 + threadIdx.x];
  __syncthreads();
  double2 *dst = c + ((size_t)r * V + i0) * 12;
  for (int q = threadIdx.x; q < nv * 12; q += 256) dst[q] = t[(q % 12) * 257 + q / 12];
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
