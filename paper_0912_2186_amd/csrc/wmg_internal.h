// Internal declarations of the gfx950 multigrid library (not installed).
//
// Layouts in device memory (all chosen for coalesced, site-fastest access):
//   fine spinor   [rhs][12][Vs]  complex (double2 / float2), component
//                 c = spin*3 + colour, lexicographic site s = x+Lx(y+Ly(z+Lz t)),
//                 Vs = fine_stride(V) (padding entries are zero)
//   gauge links   [4][9][Vs]     complex (double2 / float2 / __half2), element
//                 (mu, 3a+b) of U_mu(s)
//   coarse vector [rhs][Vc][n]   complex, n = 2 Nv dof per site ordered (chi, alpha)
//   coarse links  [Vc][9][n][n]  complex, direction d = 0 local, 1+mu forward,
//                 5+mu backward; row-major within a block
//   prolongator   [nv][Vc][bs][h2]  block-major: for null vector alpha and
//                 coarse site xh the bs fine sites of the block in lexicographic
//                 order inside the block, each with its `dof` components
//                 (12 on the fine lattice, n on a coarse one)
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stddef.h>
#include <stdint.h>

#include <functional>
#include <string>

namespace wmg {

// ---------------------------------------------------------------- complex
template <class R> struct cx {
  R re, im;
};
template <class R> __host__ __device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <class R> __host__ __device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <class R> __host__ __device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class R> __host__ __device__ __forceinline__ cx<R> operator*(R a, cx<R> b) { return {a * b.re, a * b.im}; }
// conj(a) * b
template <class R> __host__ __device__ __forceinline__ cx<R> cmulc(cx<R> a, cx<R> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
__host__ __device__ __forceinline__ float mad(float a, float b, float c) { return fmaf(a, b, c); }
__host__ __device__ __forceinline__ double mad(double a, double b, double c) { return fma(a, b, c); }
template <class R> __host__ __device__ __forceinline__ cx<R> cfma(cx<R> a, cx<R> b, cx<R> c) {  // a*b + c
  return {mad(a.re, b.re, mad(-a.im, b.im, c.re)), mad(a.re, b.im, mad(a.im, b.re, c.im))};
}
template <class R> __host__ __device__ __forceinline__ cx<R> cfmac(cx<R> a, cx<R> b, cx<R> c) {  // conj(a)*b + c
  return {mad(a.re, b.re, mad(a.im, b.im, c.re)), mad(a.re, b.im, mad(-a.im, b.re, c.im))};
}
template <class R> __host__ __device__ __forceinline__ cx<R> times_i(cx<R> a) { return {-a.im, a.re}; }
template <class R> __host__ __device__ __forceinline__ cx<R> times_mi(cx<R> a) { return {a.im, -a.re}; }
template <class R> __host__ __device__ __forceinline__ cx<R> neg(cx<R> a) { return {-a.re, -a.im}; }
template <class R> __host__ __device__ __forceinline__ cx<R> czero() { return {R(0), R(0)}; }

// storage element <-> arithmetic complex
__device__ __forceinline__ cx<double> ldc(const double2 *p) { double2 v = *p; return {v.x, v.y}; }
__device__ __forceinline__ cx<float> ldc(const float2 *p) { float2 v = *p; return {v.x, v.y}; }
__device__ __forceinline__ cx<float> ldc(const __half2 *p) {
  float2 v = __half22float2(*p);
  return {v.x, v.y};
}
__device__ __forceinline__ void stc(double2 *p, cx<double> v) { *p = make_double2(v.re, v.im); }
__device__ __forceinline__ void stc(float2 *p, cx<float> v) { *p = make_float2(v.re, v.im); }
__device__ __forceinline__ void stc(double2 *p, cx<float> v) { *p = make_double2(v.re, v.im); }
__device__ __forceinline__ void stc(float2 *p, cx<double> v) { *p = make_float2((float)v.re, (float)v.im); }
__device__ __forceinline__ void stc(__half2 *p, cx<float> v) { *p = __floats2half2_rn(v.re, v.im); }
// value as it reads back after a store to S (rounding of FP16 storage)
__device__ __forceinline__ cx<float> as_stored(const __half2 *, cx<float> v) {
  float2 r = __half22float2(__floats2half2_rn(v.re, v.im));
  return {r.x, r.y};
}
template <class S, class R> __device__ __forceinline__ cx<R> as_stored(const S *, cx<R> v) { return v; }

template <class S> struct store_traits;
template <> struct store_traits<double2> { using real = double; };
template <> struct store_traits<float2> { using real = float; };
template <> struct store_traits<__half2> { using real = float; };

// ---------------------------------------------------------------- packs
// Vector kernels move PK consecutive complex elements per lane and access so
// that every load and store is 16 bytes wide (one FP64, two FP32 or four
// FP16 complex numbers; a wider pack of a mixed-precision kernel is two
// accesses).  Vectors are hipMalloc'd and their per-rhs length is a multiple
// of PK, so every pack is aligned.
template <class S> __host__ __device__ constexpr int pack_len() { return 16 / (int)sizeof(S); }
template <class S, int PK> struct alignas(sizeof(S) * PK >= 16 ? 16 : sizeof(S) * PK) Pack {
  S v[PK];
};
template <int PK, class S, class R> __device__ __forceinline__ void ldp(const S *p, cx<R> o[PK]) {
  const Pack<S, PK> t = *reinterpret_cast<const Pack<S, PK> *>(p);
#pragma unroll
  for (int k = 0; k < PK; k++) {
    auto c = ldc(&t.v[k]);
    o[k] = {(R)c.re, (R)c.im};
  }
}
template <int PK, class S, class R> __device__ __forceinline__ void stp(S *p, const cx<R> v[PK]) {
  Pack<S, PK> t;
#pragma unroll
  for (int k = 0; k < PK; k++) stc(&t.v[k], v[k]);
  *reinterpret_cast<Pack<S, PK> *>(p) = t;
}

// ---------------------------------------------------------------- geometry
struct Geom {
  int L[4];
  long V;   // sites
  long Vs;  // site stride of fine-lattice SoA arrays (>= V, see fine_stride)
};

// Fine-lattice SoA fields keep their components fine_stride(V) sites apart
// rather than V: with V a power of two every component of a site would sit
// at the same offset modulo the cache-set period and the 12 spinor and 36
// link components of one site would compete for the same L2 sets.
__host__ __device__ __forceinline__ long fine_stride(long V) { return (V + 63) / 64 * 64 + 320; }

__host__ __device__ __forceinline__ void site_coords(const int L[4], long s, int x[4]) {
  x[0] = (int)(s % L[0]); s /= L[0];
  x[1] = (int)(s % L[1]); s /= L[1];
  x[2] = (int)(s % L[2]); s /= L[2];
  x[3] = (int)s;
}
__host__ __device__ __forceinline__ long site_index(const int L[4], const int x[4]) {
  return x[0] + (long)L[0] * (x[1] + (long)L[1] * (x[2] + (long)L[2] * x[3]));
}

// Workgroup -> tile remap so that each of the 8 XCDs (which receive
// workgroups round-robin) walks one contiguous range of tiles; neighbouring
// tiles then share that XCD's L2.
// Launch xcd_grid(ntiles) workgroups; tile xcd_tile(blockIdx.x) (skip if
// >= ntiles).
static constexpr int NXCD = 8;
__host__ __device__ __forceinline__ long xcd_grid(long ntiles) { return (ntiles + NXCD - 1) / NXCD * NXCD; }
__device__ __forceinline__ long xcd_tile(long bid, long grid) { return (bid % NXCD) * (grid / NXCD) + bid / NXCD; }

enum Prec { P64 = 0, P32 = 1, P16 = 2 };
// link-precision flag: links stored as their first two rows (SU(3) fields,
// third row rebuilt in the kernel), layout [4][6][Vs]
static constexpr int LK12 = 8;

// ---------------------------------------------------------------- errors
int set_error(int code, const char *fmt, ...);
#define WMG_HIP(call)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) return ::wmg::set_error(-3, "%s:%d %s: %s", __FILE__, __LINE__, #call, hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------- autotuner
// tune.hip: *choice = the fastest of candidates 0..ncand-1 for this key
// (searched once per process, or read from the WMG_TUNE_CACHE file); run(c)
// launches candidate c once on st and returns 0 or an error code.  The last
// launch is always run(*choice).
int tune_choice(const std::string &key, int ncand, const std::function<int(int)> &run, hipStream_t st, int *choice);
// the stored choice for key, or -1
int tune_lookup(const std::string &key);

// ---------------------------------------------------------------- kernels
// dslash.hip
int wilson_canonical(const Geom &g, const double *U, double m, const double *in, double *out, hipStream_t st);
int wilson_soa(const Geom &g, int lprec, const void *U, int sprec, double m, const void *in, void *out, int nrhs,
               hipStream_t st);
// out = [bsub -] D in; with red != nullptr also <out, in>, |out|^2 per rhs ->
// red_out[rhs * red_stride + 0..2] (red: scratch of nrhs * wilson_red_blocks * 3);
// with out32 != nullptr (FP64 spinors only) out is also written as FP32 there,
// and out may then be nullptr (FP32 copy only; the reductions stay FP64)
int wilson_soa_fused(const Geom &g, int lprec, const void *U, int sprec, double m, const void *in, void *out, int nrhs,
                     const void *bsub, double *red, double *red_out, int red_stride, hipStream_t st,
                     void *out32 = nullptr);
// out (FP32) = D in with FP32 links (lprec may carry LK12) on an FP16 input
// field (FP32 arithmetic): the inner GCR's operator on the FP16-stored
// preconditioner output.  With red, <out, dotv> (dotv an FP32 field of the
// same layout; <out, in> without it) and |out|^2 per rhs -> red_out as in
// wilson_soa_fused.
int wilson_soa_in16(const Geom &g, int lprec, const void *U, double m, const void *in, void *out, int nrhs,
                    hipStream_t st, double *red = nullptr, double *red_out = nullptr, int red_stride = 0,
                    const void *dotv = nullptr);
// Smoother variant with FP16 links and FP16 output storage: in is FP32
// (iprec P32) or FP16 (P16); out (FP16) = [b/|b| -] D in, where bsub (FP32)
// is scaled per rhs by 1/sqrt(bnrm2[rhs * bstride]) (0 where that norm is
// 0); red as in wilson_soa_fused, computed from the stored (rounded) output.
// lflags: LK12 for links stored as two rows.  With out_odd (bsub given, no
// reductions) the output goes to the half-lattice arrays out (even sites)
// and out_odd (odd sites) instead of a full-lattice field.  FP16 input with
// bsub only with out_odd.  With FP16 input the hopping sum runs in packed
// FP16 arithmetic (projection, SU(3) products, each direction's forward
// and backward terms combined), the directions summed in FP32; with FP32
// input, and the diagonal and bsub terms always, in FP32.
int wilson_soa_h16(const Geom &g, const void *U16, int iprec, double m, const void *in, void *out, int nrhs,
                   const void *bsub, const double *bnrm2, int bstride, double *red, double *red_out, int red_stride,
                   hipStream_t st, int lflags = 0, void *out_odd = nullptr);
// partials per rhs that the fused reductions of wilson_soa_fused,
// wilson_soa_h16 and hop_eo may write (the largest of their tilings)
long wilson_red_blocks(const Geom &g);
// ---- red/black (even-odd) sublattices; requires every extent even.
// Compact half-lattice arrays: site of lexicographic index s, parity p at
// index s/2 of parity p's array; fields [rhs][colour][eo_stride][spin],
// links [parity][4][NR][eo_stride].
long eo_stride(const Geom &g);
long eo_red_tiles(const Geom &g);
// out = a in_diag + b H_par(in_hop) on the sites of parity par (H: the
// hopping sum of Eq. 2.2 from the other sublattice; D_{p,1-p} = -H/2);
// with red, <out, in_diag> and |out|^2 per rhs -> red_out[rhs * stride + 0..2]
// (red: scratch of nrhs * wilson_red_blocks * 3).  Precision combinations:
// all FP64; FP16 links with FP16 in_diag and in_hop/out FP16 or FP32.
int hop_eo(const Geom &g, int lprec, const void *Ue, int par, double a, double b, int pdiag, const void *in_diag,
           int phop, const void *in_hop, int pout, void *out, int nrhs, double *red, double *red_out, int red_stride,
           hipStream_t st);
// full (full-lattice, precision phop) += d_e at the even sites and
// a in_diag + b H_odd(d_e) at the odd sites, d_e the even half-lattice field
// (precision phop): all FP64, or FP16 links and in_diag with FP32 or FP16
// d_e and FP32 full.  With ebase (FP16 d_e only: an FP16 full-lattice field)
// full = ebase + (d_e, d_o) instead, full not read; full is then FP32, or
// FP16 with pfull = P16 (sums in FP32, rounded once).
int hop_eo_add(const Geom &g, int lprec, const void *Ue, double a, double b, int pdiag, const void *in_diag,
               int phop, const void *de, void *full, int nrhs, hipStream_t st, const void *ebase = nullptr,
               int pfull = P32);
int eo_pack(const Geom &g, int pfull, const void *full, int phalf, void *ev, void *od, int nrhs, hipStream_t st);
int eo_unpack_add(const Geom &g, int pfull, void *full, int phalf, const void *ev, const void *od, int nrhs,
                  hipStream_t st);
int links_to_eo(const Geom &g, const void *U64soa, int lprec, void *Ue, hipStream_t st);
// lprec may carry LK12: only the first two rows, layout [4][6][Vs]
int links_to_soa(const Geom &g, const double *Ucanon, int lprec, void *Usoa, hipStream_t st);
// per-workgroup largest error of the 12-real reconstruction of canonical
// FP64 links (su3_recon_blocks(g) doubles)
long su3_recon_blocks(const Geom &g);
int su3_recon_err(const Geom &g, const double *Ucanon, double *part, hipStream_t st);
int spinor_to_soa(const Geom &g, const double *canon, double2 *soa, int nrhs, hipStream_t st);
int spinor_from_soa(const Geom &g, const double2 *soa, double *canon, int nrhs, hipStream_t st);

// blas.hip -- flat complex vectors [nrhs][n]
struct Reducer {
  double *partial;  // [nrhs][maxblk][32] per-workgroup partial sums
  int maxblk;
  int nrhs_max;
  bool owned;       // partial was allocated by red_init (freed by red_free)
};
int red_init(Reducer &r, int nrhs_max);
void red_free(Reducer &r);
// bytes of partials for nrhs_max right-hand sides; red_attach uses memory the
// caller owns (red_free then leaves it alone)
size_t red_bytes(int nrhs_max);
void red_attach(Reducer &r, int nrhs_max, double *partial);
// out[rhs*stride + 0..1] = <x,y> (re, im)
int dot(Reducer &R, int prec, const void *x, const void *y, long n, int nrhs, double *out, int out_stride, hipStream_t st);
int norm2(Reducer &R, int prec, const void *x, long n, int nrhs, double *out, int out_stride, hipStream_t st);
// out[rhs * out_stride] = sum_b part[rhs * nblk + b], fixed order (one workgroup per rhs)
int sum_partials(const double *part, long nblk, int nrhs, double *out, int out_stride, hipStream_t st);
// out[rhs*stride+0..1] = <x,y>, out[rhs*stride+2] = |x|^2
int dot_norm(Reducer &R, int prec, const void *x, const void *y, long n, int nrhs, double *out, int out_stride,
             hipStream_t st);
int copy(int pdst, void *dst, int psrc, const void *src, long n, int nrhs, hipStream_t st);
int zero(int prec, void *x, long n, int nrhs, hipStream_t st);
// y[rhs] += sgn * a[rhs] x[rhs]   (a complex, read from device: a[rhs*astride + 0..1])
int caxpy_dev(int prec, const double *a, int astride, double sgn, const void *x, void *y, long n, int nrhs,
              hipStream_t st);
// y = x + sgn*a*y   (xpay)
int cxpay_dev(int prec, const void *x, const double *a, int astride, double sgn, void *y, long n, int nrhs,
              hipStream_t st);
// y[rhs] = sum_j c[rhs][j] x_j[rhs]  + (accumulate ? y : 0),  x_j given by pointer list (device array)
int multi_caxpy(int py, void *y, int px, const void *const *xs_dev, int k, const double *c, int cstride, double sgn,
                int accumulate, long n, int nrhs, hipStream_t st);
// y = a x + b y (host scalars)
int axpby(int prec, double a, const void *x, double b, void *y, long n, int nrhs, hipStream_t st);
// out[rhs][j] = <x_j, y> for j < k
int multi_dot(Reducer &R, int prec, const void *const *xs_dev, int k, const void *y, long n, int nrhs, double *out,
              int out_stride, hipStream_t st);
// GCR Gram-Schmidt pass against unnormalised w_j (see blas.hip)
int gcr_project(Reducer &R, int prec, int pass, const void *const *W, int k, void *w, const void *r, const double *d,
                int dstride, const double *wn2, int wstride, double *beta, int bstride, int kcol, long n, int nrhs,
                double *out, int out_stride, hipStream_t st);
// y -= a x and |y|^2 -> out
int caxpy_norm(Reducer &R, int prec, const double *a, int astride, const void *x, void *y, long n, int nrhs,
               double *out, int out_stride, hipStream_t st);
// y = a - b
int csub(int prec, const void *a, const void *b, void *y, long n, int nrhs, hipStream_t st);
// x *= 1/sqrt(nrm2[rhs])  (nrm2 device)
int scale_inv_sqrt(int prec, void *x, const double *nrm2, int stride, long n, int nrhs, hipStream_t st);
// x *= sqrt(nrm2[rhs])
int scale_sqrt(int prec, void *x, const double *nrm2, int stride, long n, int nrhs, hipStream_t st);
int sigma3(int prec, void *x, long nsite, int dof, int nrhs, hipStream_t st);

// transfer.hip
// count vectors; fine (SoA): component stride Vs, vector stride 12*Vs;
// coarse (AoS): vector stride nsite*dof
int start_vectors(long nsite, int dof, uint64_t seed, int lvl, int alpha0, int count, double2 *out_soa_or_aos,
                  int fine_soa, long Vs, hipStream_t st);
// ns: parts of the per-site components in the blocking (2 chiralities; 4
// Dirac spins on the fine level), coarse dof ns * nv ordered (part, vector)
// vectors a0 .. nv-1 (the earlier columns of P are kept: each vector is
// orthogonalised against the ones before it only)
int block_orthonormalize(const Geom &g, int dof, const int b[4], int nv, const double2 *vecs, int fine_soa,
                         double2 *P, int *fail_dev, hipStream_t st, int ns = 2, int a0 = 0);
// rn2 != nullptr (|fine|^2 per rhs at stride rstride): the fine-level
// matrix-core restriction with FP16 products (transfer.hip)
int restrict_op(const Geom &g, int dof, const int b[4], int nv, int pprec, const void *P, const float *Pscale,
                int vprec, const void *fine, int fine_soa, void *coarse, int nrhs, hipStream_t st, int ns = 2,
                const double *rn2 = nullptr, int rstride = 0);
// cpart != nullptr (COARSE_H_PART floats per rhs, nrhs <= COARSE_H_MAXRHS):
// the fine-level matrix-core prolongation with FP16 products when Nv % 8 == 0
// out16: the fine field in FP16 (FP16 products only; prolong_h_supported)
int prolong_op(const Geom &g, int dof, const int b[4], int nv, int pprec, const void *P, const float *Pscale,
               int vprec, const void *coarse, void *fine, int fine_soa, int nrhs, hipStream_t st, int ns = 2,
               float *cpart = nullptr, bool out16 = false);
bool prolong_h_supported(const Geom &g, int dof, const int b[4], int nv, int pprec, int vprec, int fine_soa, int ns);
int P_convert(long count, const double2 *P64, int pprec, void *Pout, float *scale, int dof, hipStream_t st);
int P_convert_half(long nsites_total, int bs, int dof, int fine, const double2 *P64, __half2 *Ph, float *scale,
                   hipStream_t st);
int P_block_to_vector(const Geom &g, int dof, const int b[4], int nv, const double2 *P, double2 *vec, int fine_soa,
                      hipStream_t st);

// coarse.hip
int coarse_build(const Geom &g, int fine_kind, int dof, const void *U64soa, double m, const double2 *Yf, const int b[4],
                 int nv, const double2 *P, double2 *Yc, double2 *work, hipStream_t st, int ns = 2);
// One step of the adaptive setup's rebuild: with the first k - 1 columns of
// every part already in Ys (blocks of leading dimension ns * nld), build the
// columns of vector k - 1, mirror them into its rows (gamma_5-hermiticity of
// the coarse operator) and write the compact blocks of the first k vectors
// to Yc.  The prolongator's first k - 1 vectors must be those Ys was built
// from (block Gram-Schmidt leaves earlier vectors unchanged).
int coarse_build_next(const Geom &g, int fine_kind, int dof, const void *U64soa, double m, const double2 *Yf,
                      const int b[4], int k, int nld, const double2 *P, double2 *Ys, double2 *Yc, hipStream_t st,
                      int ns = 2);
int coarse_apply(const Geom &gc, int n, int yprec, const void *Y, int vprec, const void *in, void *out, int dagger,
                 int nrhs, hipStream_t st);
int coarse_shift_diag(long Vc, int n, double2 *Y, double dm, hipStream_t st);
int coarse_convert(long count, const double2 *Y64, int yprec, void *Yout, hipStream_t st);
int coarse_transpose(long nblk, int n, const double2 *a, double2 *b, hipStream_t st);
// multi-RHS FP32 coarse stencil on the matrix cores (links pre-swizzled)
int coarse_to_mfma(long Vc, int n, const double2 *Y64, float *Ym, hipStream_t st);
size_t coarse_mfma_floats(long Vc, int n);
int coarse_apply_mfma(const Geom &gc, int n, const float *Ym, const float2 *in, float2 *out, int dagger, int nrhs,
                      hipStream_t st, double *npart = nullptr, bool *fused = nullptr);
// the same stencil with the swizzled links stored in FP16, one FP32 scale per
// (site, direction) block (its largest |entry|); FP32 arithmetic
int coarse_to_mfma16(long Vc, int n, const double2 *Y64, __half *Yh, float *Ysc, hipStream_t st);
size_t coarse_mfma_halfs(long Vc, int n);
// With npart != nullptr the kernels that support it (n = 32, 40, 48, 64) also
// write |out|^2 of every (rhs, site) to npart[rhs * Vc + site] and set
// *fused (sum them with sum_partials); otherwise *fused = false.  The same
// holds for coarse_apply_mfma above.
// With bpart != nullptr (scratch of COARSE_H_PART floats per rhs, nrhs <=
// COARSE_H_MAXRHS) and n = 32, 48 or 64 the products are FP16
// (v_mfma_f32_16x16x16f16) on the neighbour vectors scaled by the link block
// scale and one power-of-two scale per rhs, accumulated in FP32.
constexpr int COARSE_H_PART = 32;
constexpr int COARSE_H_MAXRHS = 64;
// partial maxima of |re|, |im| of each rhs's vector (len complex per rhs):
// COARSE_H_PART per rhs into part
int rhs_absmax(const float2 *v, long len, int nrhs, float *part, hipStream_t st);
int coarse_apply_mfma16(const Geom &gc, int n, const __half *Yh, const float *Ysc, const float2 *in, float2 *out,
                        int dagger, int nrhs, hipStream_t st, double *npart = nullptr, bool *fused = nullptr,
                        float *bpart = nullptr);

}  // namespace wmg
