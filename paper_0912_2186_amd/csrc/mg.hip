// Adaptive multigrid engine and C ABI (arXiv:0912.2186, Sec. 2-3).
//
// Host code drives device kernels on one HIP stream per context.  Solver
// scalars (dot products, step lengths, masks) live in device memory and are
// consumed by the kernels that need them; the host reads back one residual
// norm per outer GCR iteration and a convergence flag every few coarse CGNR
// iterations.
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <thread>
#include <map>
#include <tuple>
#include <vector>

#include "wmg_internal.h"
#include "../../include/wmg.h"

namespace wmg {

static thread_local char g_err[512] = "";

int set_error(int code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}


static constexpr int KMAX = 16;
static size_t csize(int prec) { return prec == P64 ? 16 : (prec == P16 ? 4 : 8); }

// ------------------------------------------------------------ scalar kernels
// MR step: alpha = <q,s>/|q|^2 (red[rhs*4 + 0..2]); e += alpha s; s -= alpha q
template <class S>
__global__ void k_mr_update(const double *__restrict__ red, S *__restrict__ e, S *__restrict__ s,
                            const S *__restrict__ q, long n) {
  using R = typename store_traits<S>::real;
  int rhs = blockIdx.y;
  const double *rd = red + rhs * 4;
  double qq = rd[2];
  cx<R> a = qq > 0 ? cx<R>{(R)(rd[0] / qq), (R)(rd[1] / qq)} : czero<R>();
  size_t off = (size_t)rhs * n;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
    auto sv = ldc(s + off + i);
    auto qv = ldc(q + off + i);
    auto ev = ldc(e + off + i);
    stc(e + off + i, cfma(a, sv, ev));
    stc(s + off + i, cfma(neg(a), qv, sv));
  }
}

// MR with the solution update deferred (fine level): step k only forms the
// next residual s_{k+1} = s_k - alpha_k q_k; after the last step
// e += sum_k alpha_k s_k in one pass.  alpha_k = <q_k,s_k>/|q_k|^2 from
// red[(k*64 + rhs)*4 + 0..2].
template <class R> __device__ __forceinline__ cx<R> mr_alpha(const double *red, int k, int rhs) {
  const double *rd = red + ((size_t)k * 64 + rhs) * 4;
  double qq = rd[2];
  return qq > 0 ? cx<R>{(R)(rd[0] / qq), (R)(rd[1] / qq)} : czero<R>();
}
template <class S>
__global__ void k_mr_next(const double *__restrict__ red, int k, const S *__restrict__ s, const S *__restrict__ q,
                          S *__restrict__ snext, long n) {
  using R = typename store_traits<S>::real;
  constexpr int PK = pack_len<S>();
  int rhs = blockIdx.y;
  cx<R> a = neg(mr_alpha<R>(red, k, rhs));
  size_t off = (size_t)rhs * n;
  const long np = n / PK;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < np; i += (long)gridDim.x * 256) {
    cx<R> qv[PK], sv[PK];
    ldp<PK>(q + off + i * PK, qv);
    ldp<PK>(s + off + i * PK, sv);
#pragma unroll
    for (int e = 0; e < PK; e++) sv[e] = cfma(a, qv[e], sv[e]);
    stp<PK>(snext + off + i * PK, sv);
  }
}
struct MrVecs {
  const void *s[4];
};
// e (+)= sum_k alpha_k s_k; ACC = 0 overwrites e
template <class S, class SS = S, int ACC = 1>
__global__ void k_mr_accum(const double *__restrict__ red, int nsteps, MrVecs v, S *__restrict__ e, long n) {
  using R = typename store_traits<S>::real;
  constexpr int PK = pack_len<S>() > pack_len<SS>() ? pack_len<S>() : pack_len<SS>();
  int rhs = blockIdx.y;
  cx<R> a[4];
#pragma unroll
  for (int k = 0; k < 4; k++) a[k] = k < nsteps ? mr_alpha<R>(red, k, rhs) : czero<R>();
  size_t off = (size_t)rhs * n;
  const long np = n / PK;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < np; i += (long)gridDim.x * 256) {
    cx<R> acc[PK];
    if (ACC) {
      ldp<PK>(e + off + i * PK, acc);
    } else {
#pragma unroll
      for (int q = 0; q < PK; q++) acc[q] = czero<R>();
    }
#pragma unroll
    for (int k = 0; k < 4; k++)
      if (k < nsteps) {
        cx<R> sv[PK];
        ldp<PK>((const SS *)v.s[k] + off + i * PK, sv);
#pragma unroll
        for (int q = 0; q < PK; q++) acc[q] = cfma(a[k], sv[q], acc[q]);
      }
    stp<PK>(e + off + i * PK, acc);
  }
}

// CG: alpha = act ? ss/uu : 0; x += alpha p; r -= alpha u
// and the workgroup's part of |r|^2 (after the update) into
// part[rhs * gridDim.x + blockIdx.x]
template <class S>
__global__ void __launch_bounds__(256) k_cg_step1(const double *__restrict__ cg, int ssoff, S *__restrict__ x,
                                                 S *__restrict__ r, const S *__restrict__ p, const S *__restrict__ u,
                                                 long n, int nrhs, double *__restrict__ part) {
  using R = typename store_traits<S>::real;
  int rhs = blockIdx.y;
  const double *c = cg + rhs * 8;
  double uu = c[0], ss = c[ssoff], act = c[5];
  R a = (act > 0 && uu > 0) ? (R)(ss / uu) : R(0);
  size_t off = (size_t)rhs * n;
  double q = 0;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
    auto rv = ldc(r + off + i);
    if (a != R(0)) {
      auto pv = ldc(p + off + i), uv = ldc(u + off + i);
      stc(x + off + i, ldc(x + off + i) + a * pv);
      rv = rv - a * uv;
      stc(r + off + i, rv);
    }
    q += (double)rv.re * rv.re + (double)rv.im * rv.im;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) q += __shfl_down(q, o, 64);
  __shared__ double sh[4];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = q;
  __syncthreads();
  if (threadIdx.x == 0) part[(size_t)rhs * gridDim.x + blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// CG: p = s + beta p, beta = ss_new/ss_old, only while active
template <class S>
__global__ void k_cg_step2(const double *__restrict__ cg, int newoff, int oldoff, const S *__restrict__ s,
                           S *__restrict__ p, long n) {
  using R = typename store_traits<S>::real;
  int rhs = blockIdx.y;
  const double *c = cg + rhs * 8;
  if (!(c[5] > 0)) return;
  R be = c[oldoff] > 0 ? (R)(c[newoff] / c[oldoff]) : R(0);
  size_t off = (size_t)rhs * n;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256)
    stc(p + off + i, ldc(s + off + i) + be * ldc(p + off + i));
}

// cg layout per rhs (8 doubles): 0 uu, 1 ss[0], 2 ss[1], 3 rr, 4 bb, 5 active, 6 iters, 7 tol^2
__global__ void k_cg_init(double *cg, int nrhs, double tol2, const double *mask) {
  int r = threadIdx.x;
  if (r >= nrhs) return;
  double *c = cg + r * 8;
  c[5] = (c[4] > 0 && (!mask || mask[r] > 0)) ? 1.0 : 0.0;
  c[6] = 0;
  c[7] = tol2;
}
__global__ void k_cg_check(double *cg, int nrhs, int *alldone) {
  int r = threadIdx.x;
  __shared__ int any;
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  if (r < nrhs) {
    double *c = cg + r * 8;
    if (c[5] > 0) {
      c[6] += 1;
      if (c[3] <= c[7] * c[4]) c[5] = 0;
      else atomicOr(&any, 1);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) *alldone = any ? 0 : 1;
}

// GCR coefficient bookkeeping.  gcr layout per rhs (stride GS doubles):
//   beta[K][K][2] | wn2[K] (|w_k|^2 of the unnormalised basis) | alpha[K][2] |
//   c[K][2] | tmp[2K] (first-pass projections) | tmp2[2K] (second pass)
constexpr int GK = KMAX;
constexpr int G_BETA = 0, G_GAMMA = G_BETA + GK * GK * 2, G_ALPHA = G_GAMMA + GK, G_C = G_ALPHA + GK * 2,
              G_TMP = G_C + GK * 2, G_TMP2 = G_TMP + 2 * GK, GS = G_TMP2 + 2 * GK + 8;
// wn2[k] = |w_k|^2; alpha_k = <w_k, r>/|w_k|^2 for participating rhs, else 0
// (red holds <w_k, r> in slots 0,1 and |w_k|^2 in slot 2)
__global__ void k_gcr_alpha2(double *g, const double *red, const double *mask, int k, int nrhs) {
  int r = threadIdx.x;
  if (r >= nrhs) return;
  double q = red[r * 4 + 2];
  g[r * GS + G_GAMMA + k] = q;
  bool ok = mask[r] > 0 && q > 0;
  g[r * GS + G_ALPHA + 2 * k] = ok ? red[r * 4] / q : 0.0;
  g[r * GS + G_ALPHA + 2 * k + 1] = ok ? red[r * 4 + 1] / q : 0.0;
}
// back substitution for A z_k = w_k + sum_{j<k} beta_jk w_j:
//   c_j = alpha_j - sum_{i>j} beta_ji c_i   (c_j = 0 where w_j vanished)
__global__ void k_gcr_trisolve2(double *g, int k, int nrhs) {
  int r = threadIdx.x;
  if (r >= nrhs) return;
  double *G = g + r * GS;
  for (int j = k - 1; j >= 0; j--) {
    double tr = G[G_ALPHA + 2 * j], ti = G[G_ALPHA + 2 * j + 1];
    for (int i = j + 1; i < k; i++) {
      double br = G[G_BETA + (j * GK + i) * 2], bi = G[G_BETA + (j * GK + i) * 2 + 1];
      double cr = G[G_C + 2 * i], ci = G[G_C + 2 * i + 1];
      tr -= br * cr - bi * ci;
      ti -= br * ci + bi * cr;
    }
    bool ok = G[G_GAMMA + j] > 0;
    G[G_C + 2 * j] = ok ? tr : 0.0;
    G[G_C + 2 * j + 1] = ok ? ti : 0.0;
  }
}

// one lane per pack of S (pack_len<S>() complex numbers; 1 for kernels that
// walk single elements): more loads in flight than a grid-stride loop
template <class S> static dim3 grid_for(long n, int nrhs) {
  long b = (n / pack_len<S>() + 255) / 256;
  if (b > (1L << 30) / 256) b = (1L << 30) / 256;
  if (b < 1) b = 1;
  return dim3((unsigned)b, nrhs);
}

}  // namespace wmg

using namespace wmg;

// ------------------------------------------------------------ context
enum { VR, VE, VT, VE2, VS, VQ, VCR, VCS, VCP, VCU, VX, VS1, VS2, VS3,
       // red/black smoother: sublattice residuals, MR iterates, corrections
       VH0, VH1, VH2, VH3, VHQ, VHT, VHSE, VHSO, VHDE, VHDO,
       VEH,  // FP16 copy of the prolonged correction (red/black smoother of the mixed cycle)
       NVW };

struct Level {
  Geom g;
  int dof = 12;
  bool fine = true;
  long n = 0;        // complex numbers per rhs at the current Nv of the level above
  long n_alloc = 0;  // ... at its largest Nv (allocation size)
  // fine operator
  void *U[3] = {nullptr, nullptr, nullptr};  // P64 / P32 / P16 SoA, whole links [4][9][Vs]
  void *Uk[3] = {nullptr, nullptr, nullptr}; // the same as two rows [4][6][Vs] (SU(3) fields)
  int lk = 0;                                // LK12 when the Dslash uses Uk
  void *Ue[3] = {nullptr, nullptr, nullptr}; // red/black copies [parity][4][NR][eo_stride] (built on first use)
  double m = 0;
  // coarse operator (internal layout)
  double2 *Y64 = nullptr;
  float2 *Y32 = nullptr;  // FP32 copy for the vector-FMA stencil (n > 64)
  float *Ym = nullptr;    // FP32 copy swizzled for the MFMA stencil (n <= 64)
  __half *Ymh = nullptr;  // ... or its FP16 copy with one scale per (site, direction)
  float *Ymsc = nullptr;
  int dof_max = 0;
  // transfer to level+1
  int b[4] = {1, 1, 1, 1};
  int ns = 2;  // parts per site in the blocking: 2 chiralities, or 4 spins (fine level, WMG_SPIN_SPLIT)
  int nv = 0, nv_max = 0;
  double2 *vecs = nullptr;  // null vectors, level vector layout, FP64
  double2 *P64 = nullptr;
  float2 *P32 = nullptr;
  __half2 *P16 = nullptr;
  float *Ps = nullptr;
  // work vectors: [prec][name] each [cap][n_alloc], cap = largest nrhs asked for
  void *w[3][NVW] = {};  // work vectors by storage precision (P64, P32, P16)
  int w_cap[3][NVW] = {};
};

struct GcrBuf {
  int prec = P64;  // inner precision
  int nrhs = 0;
  long n = 0;
  void *z[KMAX] = {}, *wv[KMAX] = {};
  void **zdev = nullptr, **wdev = nullptr;  // device arrays of the pointers
  void *rin = nullptr;                      // inner residual (aliases r64 in FP64 mode)
  double2 *x64 = nullptr, *r64 = nullptr, *b64 = nullptr, *t64 = nullptr;
  // storage precision the z[k] last held (-1: as allocated, zero); the
  // vector kernels sweep whole arrays, so the site padding of the other
  // view is cleared when it changes
  int zfmt = -1;
};

// links the fine operator reads at precision lp, and the precision code
// (with LK12 when they are stored as two rows)
static inline const void *fine_links(const Level &L, int lp) { return L.lk ? L.Uk[lp] : L.U[lp]; }
static inline int fine_lcode(const Level &L, int lp) { return lp | L.lk; }
// complex numbers of link data per site the fine operator reads
static inline double fine_link_cx(const Level &L) { return L.lk ? 24.0 : 36.0; }

struct wmg_ctx {
  wmg_params p;
  int nl = 2;       // levels of the final hierarchy
  int nl_cur = 2;   // levels in use (the setup's trial schemes use fewer)
  Level lv[3];
  hipStream_t st = nullptr;
  Reducer red{};
  double *dsc = nullptr;  // device scalars
  double *red_out = nullptr;
  double *mr_red = nullptr;  // fused MR step reductions, [step][rhs][4]
  double *cyc_nrm = nullptr;  // |r|^2 of the cycle input per rhs, [rhs][4]
  bool verbose = false;       // WMG_VERBOSE set: one stderr line per setup vector
  double *cg = nullptr;
  double *gcr = nullptr;
  double *mask = nullptr;
  double *dred = nullptr;  // per-workgroup partials of the fused Dslash reductions
  double *cpart = nullptr;  // per-(rhs, site or workgroup) partials of fused coarse norms
  size_t cpart_cap = 0;
  float *bpart = nullptr;   // per-rhs partial maxima for the FP16 products of the coarse stencil
  int *flag = nullptr;
  double *hbuf = nullptr;  // pinned host mirror
  GcrBuf gb[2][2];         // [level 0 / level 1][FP64 / FP32 inner precision]
  // coarse CGNR iteration blocks captured as HIP graphs (WMG_GRAPHS): key ->
  // (times seen, block of 4 iterations minus the last second half, that half)
  struct CgGraph {
    int seen = 0;
    bool failed = false;
    hipGraphExec_t blk = nullptr, tail = nullptr;
  };
  std::map<std::vector<uintptr_t>, CgGraph> cg_graphs;
  std::vector<int> last_iters;
  double setup_s = 0;
  // solve statistics
  long st_fine = 0, st_fine64 = 0, st_coarse = 0, st_rel = 0;
  // batch
  std::vector<wmg_ctx *> batch;
  // per-kernel-class event timing (mg_profile)
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<int> ev_kind;  // kind of each recorded pair
  std::vector<double> ev_bytes;
  int ev_used = 0;           // pairs recorded and not yet resolved
  double prof_ms[8] = {0}, prof_bytes[8] = {0};
  long prof_n[8] = {0};
};

// kernel classes timed by mg_profile
enum { K_DSLASH_CYCLE = 0, K_DSLASH_OUTER32 = 1, K_DSLASH_64 = 2, K_COARSE32 = 3, K_COARSE64 = 4, K_RESTRICT = 5,
       K_PROLONG = 6, K_DSLASH_RES = 7, K_NKIND = 8 };
static const int EV_CAP = 2048;

static int prof_resolve(wmg_ctx *c) {
  if (!c->ev_used) return 0;
  WMG_HIP(hipStreamSynchronize(c->st));
  for (int i = 0; i < c->ev_used; i++) {
    float t = 0;
    WMG_HIP(hipEventElapsedTime(&t, c->ev_pool[2 * i], c->ev_pool[2 * i + 1]));
    int k = c->ev_kind[i];
    c->prof_ms[k] += t;
    c->prof_bytes[k] += c->ev_bytes[i];
    c->prof_n[k]++;
  }
  c->ev_used = 0;
  return 0;
}

// record the start event of a timed launch; returns the pair slot or -1
static int prof_begin(wmg_ctx *c, int kind, double bytes) {
  if (!c->prof) return -1;
  if (c->ev_pool.empty()) {
    c->ev_pool.resize(2 * EV_CAP);
    c->ev_kind.resize(EV_CAP);
    c->ev_bytes.resize(EV_CAP);
    for (auto &e : c->ev_pool)
      if (hipEventCreate(&e) != hipSuccess) return -1;
  }
  if (c->ev_used == EV_CAP && prof_resolve(c)) return -1;
  int i = c->ev_used++;
  c->ev_kind[i] = kind;
  c->ev_bytes[i] = bytes;
  (void)hipEventRecord(c->ev_pool[2 * i], c->st);
  return i;
}
static void prof_end(wmg_ctx *c, int slot) {
  if (slot >= 0) (void)hipEventRecord(c->ev_pool[2 * slot + 1], c->st);
}

static int dalloc(void **p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) return set_error(WMG_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  // zero-filled: the site padding of fine-lattice fields must read as zero
  // in every vector kernel that sweeps whole arrays
  // (on the default stream, waited for here: the contexts' own streams are
  // non-blocking, so nothing else orders their later kernels after the fill)
  e = hipMemset(*p, 0, bytes);
  if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  if (e != hipSuccess) return set_error(WMG_EHIP, "hipMemset: %s", hipGetErrorString(e));
  return 0;
}
#define TRY(x)            \
  do {                    \
    int rc_ = (x);        \
    if (rc_) return rc_;  \
  } while (0)

static int sync(wmg_ctx *c) {
  WMG_HIP(hipStreamSynchronize(c->st));
  return 0;
}

// Low-precision (and, for SU(3) fields, two-row) copies of the fine links.
// The two-row format is used when every link's third row equals
// conj(row0 x row1) to 1e-12 (e.g. links exp(i eps H) with traceless
// Hermitian H, and their gauge transforms) and force18 is false; the FP64
// whole links stay for the Galerkin build.
static int fine_link_format(wmg_ctx *c, Level &F, const double *U, bool force18) {
  bool c12 = false;
  if (!force18) {
    const long nb = su3_recon_blocks(F.g);
    double *part = nullptr;
    TRY(dalloc((void **)&part, sizeof(double) * nb));
    std::vector<double> h(nb);
    int rc = su3_recon_err(F.g, U, part, c->st);
    if (!rc && hipMemcpyAsync(h.data(), part, sizeof(double) * nb, hipMemcpyDeviceToHost, c->st) != hipSuccess)
      rc = set_error(WMG_EHIP, "link check read-back");
    if (!rc) rc = sync(c);
    (void)hipFree(part);
    TRY(rc);
    double e = 0;
    for (double v : h) e = v > e ? v : e;
    c12 = e <= 1e-12;  // NaN fails too
  }
  const size_t cs[3] = {16, 8, 4};
  for (int lp = P64; lp <= P16; lp++) {
    if (c12) {
      TRY(dalloc(&F.Uk[lp], cs[lp] * 24 * (size_t)F.g.Vs));
      TRY(links_to_soa(F.g, U, lp | LK12, F.Uk[lp], c->st));
    } else if (lp != P64) {
      TRY(dalloc(&F.U[lp], cs[lp] * 36 * (size_t)F.g.Vs));
      TRY(links_to_soa(F.g, U, lp, F.U[lp], c->st));
    }
  }
  F.lk = c12 ? LK12 : 0;
  return 0;
}

// work vector `name` of level l for nrhs right-hand sides (grown on demand;
// a solve uses one nrhs throughout, so pointers stay valid within it)
static int level_vec(wmg_ctx *c, int l, int prec, int name, void **out, int nrhs) {
  Level &L = c->lv[l];
  int pi = prec == P64 ? 0 : (prec == P16 ? 2 : 1);
  if (L.w_cap[pi][name] < nrhs) {
    if (L.w[pi][name]) (void)hipFree(L.w[pi][name]);
    L.w[pi][name] = nullptr;
    L.w_cap[pi][name] = 0;
    TRY(dalloc(&L.w[pi][name], csize(prec) * (size_t)L.n_alloc * nrhs));
    L.w_cap[pi][name] = nrhs;
  }
  *out = L.w[pi][name];
  return 0;
}

// ------------------------------------------------------------ operators
// op(level, prec, in, out, nrhs, lowlinks): fine Wilson (links P64 / P32 /
// P16 when lowlinks) or coarse stencil.
static int cpart_get(wmg_ctx *c, size_t n, double **p) {
  if (c->cpart_cap < n) {
    if (c->cpart) (void)hipFree(c->cpart);
    c->cpart = nullptr;
    c->cpart_cap = 0;
    TRY(dalloc((void **)&c->cpart, sizeof(double) * n));
    c->cpart_cap = n;
  }
  *p = c->cpart;
  return 0;
}

// With nrm_out, |out|^2 per rhs -> nrm_out[rhs * nrm_stride] as well (fused
// into the multi-RHS coarse stencil where it supports it).
static int apply_op(wmg_ctx *c, int l, int prec, const void *in, void *out, int nrhs, bool lowlinks, int dagger = 0,
                    double *nrm_out = nullptr, int nrm_stride = 0) {
  Level &L = c->lv[l];
  if (L.fine) {
    int lp = prec == P64 ? P64 : (lowlinks ? P16 : P32);
    if (dagger) return set_error(-1, "fine adjoint not used");
    c->st_fine++;
    if (prec == P64) c->st_fine64++;
    // algorithmic bytes: 4 links per site + one spinor in and out per rhs
    double lb = lp == P64 ? 16 : (lp == P32 ? 8 : 4), sb = prec == P64 ? 16 : 8;
    int kind = prec == P64 ? K_DSLASH_64 : (lowlinks ? K_DSLASH_CYCLE : K_DSLASH_OUTER32);
    int slot = prof_begin(c, kind, (double)L.g.V * (fine_link_cx(L) * lb + 24.0 * sb * nrhs));
    int rc = wilson_soa(L.g, fine_lcode(L, lp), fine_links(L, lp), prec, L.m, in, out, nrhs, c->st);
    prof_end(c, slot);
    TRY(rc);
    return nrm_out ? norm2(c->red, prec, out, L.n, nrhs, nrm_out, nrm_stride, c->st) : 0;
  }
  int n = L.dof;
  // algorithmic bytes: links once (FP64 / FP32 complex, or FP16 + scales)
  // and the in and out vectors of every rhs
  double yb = prec == P64 ? 16 : (prec == P32 && L.Ymh ? 4 : 8), vb = prec == P64 ? 16 : 8;
  int slot = prof_begin(c, prec == P64 ? K_COARSE64 : K_COARSE32,
                        (double)L.g.V * (9.0 * n * n * yb + 2.0 * n * vb * nrhs));
  int rc;
  bool fused = false;
  double *npart = nullptr;
  if (nrm_out && prec == P32 && (L.Ymh || L.Ym)) TRY(cpart_get(c, (size_t)nrhs * L.g.V, &npart));
  if (prec == P32 && L.Ymh)
    rc = coarse_apply_mfma16(L.g, n, L.Ymh, L.Ymsc, (const float2 *)in, (float2 *)out, dagger, nrhs, c->st, npart,
                             &fused,
                             (c->p.flags & WMG_COARSE_B32) || nrhs > COARSE_H_MAXRHS ? nullptr : c->bpart);
  else if (prec == P32 && L.Ym)
    rc = coarse_apply_mfma(L.g, n, L.Ym, (const float2 *)in, (float2 *)out, dagger, nrhs, c->st, npart, &fused);
  else
    rc = coarse_apply(L.g, n, prec, prec == P64 ? (const void *)L.Y64 : (const void *)L.Y32, prec, in, out, dagger,
                      nrhs, c->st);
  prof_end(c, slot);
  TRY(rc);
  if (!nrm_out) return 0;
  if (fused) return sum_partials(npart, L.g.V, nrhs, nrm_out, nrm_stride, c->st);
  return norm2(c->red, prec, out, L.n, nrhs, nrm_out, nrm_stride, c->st);
}

// algorithmic bytes of one transfer: P once (plus FP16 scales) and the fine
// vectors of every rhs (coarse vectors are negligible)
static double transfer_bytes(const Level &L, int prec, int nrhs) {
  double pb = prec == P64 ? 16 : 4, vb = prec == P64 ? 16 : 8;
  double b = (double)L.nv * L.n * pb + (double)L.n * vb * nrhs;
  if (prec != P64) b += 4.0 * L.nv * L.g.V;
  return b;
}
// rn2: |fine|^2 per rhs (device, stride 4) for FP16 products on the fine
// level of the mixed cycle (nullptr, or WMG_COARSE_B32: FP32 products)
static int transfer_restrict(wmg_ctx *c, int l, int prec, const void *fine, void *coarse, int nrhs,
                             const double *rn2 = nullptr) {
  Level &L = c->lv[l];
  int pp = prec == P64 ? P64 : P16;
  const void *P = prec == P64 ? (const void *)L.P64 : (const void *)L.P16;
  if (prec != P32 || !L.fine || (c->p.flags & WMG_COARSE_B32)) rn2 = nullptr;
  int slot = l == 0 ? prof_begin(c, K_RESTRICT, transfer_bytes(L, prec, nrhs)) : -1;
  int rc = restrict_op(L.g, L.dof, L.b, L.nv, pp, P, L.Ps, prec, fine, L.fine ? 1 : 0, coarse, nrhs, c->st, L.ns,
                       rn2, 4);
  prof_end(c, slot);
  return rc;
}
// on the fine level of the mixed cycle with FP16 products (per-rhs scales
// from partial maxima in c->bpart) unless WMG_COARSE_B32
static bool prolong16_ok(wmg_ctx *c, int l, int nrhs);
static int transfer_prolong(wmg_ctx *c, int l, int prec, const void *coarse, void *fine, int nrhs,
                            bool out16 = false) {
  Level &L = c->lv[l];
  int pp = prec == P64 ? P64 : P16;
  const void *P = prec == P64 ? (const void *)L.P64 : (const void *)L.P16;
  float *cpart = prec == P32 && L.fine && c->bpart && nrhs <= COARSE_H_MAXRHS && !(c->p.flags & WMG_COARSE_B32)
                     ? c->bpart
                     : nullptr;
  int slot = l == 0 ? prof_begin(c, K_PROLONG, transfer_bytes(L, prec, nrhs)) : -1;
  if (out16 && !(cpart && prolong16_ok(c, l, nrhs))) return set_error(-1, "prolong: no FP16 output here");
  int rc = prolong_op(L.g, L.dof, L.b, L.nv, pp, P, L.Ps, prec, coarse, fine, L.fine ? 1 : 0, nrhs, c->st, L.ns,
                      cpart, out16);
  prof_end(c, slot);
  return rc;
}

// the fine-level prolongation of the mixed cycle can write FP16 (FP16
// products enabled, Nv a multiple of 8, the blocking of the MFMA kernel)
static bool prolong16_ok(wmg_ctx *c, int l, int nrhs) {
  Level &L = c->lv[l];
  return l == 0 && L.fine && c->bpart && nrhs <= COARSE_H_MAXRHS && !(c->p.flags & WMG_COARSE_B32) &&
         prolong_h_supported(L.g, L.dof, L.b, L.nv, P16, P32, 1, L.ns);
}

// fine operator with the smoother's fusions: out = [bsub -] D in, and with
// reduce also <out, in>, |out|^2 -> red_out (cycle links)
static int fine_apply_fused(wmg_ctx *c, int prec, const void *in, void *out, int nrhs, const void *bsub, bool reduce,
                            double *red_dst = nullptr, void *out32 = nullptr) {
  Level &L = c->lv[0];
  int lp = prec == P64 ? P64 : P16;
  c->st_fine++;
  if (prec == P64) c->st_fine64++;
  double lb = lp == P64 ? 16 : 4, sb = prec == P64 ? 16 : 8;
  // input, bsub, output and its FP32 copy
  const double vb = ((bsub ? 24.0 : 12.0) * sb + (out ? 12.0 * sb : 0.0) + (out32 ? 96.0 : 0.0)) * nrhs;
  int slot = prof_begin(c, prec == P64 ? K_DSLASH_64 : (bsub ? K_DSLASH_RES : K_DSLASH_CYCLE),
                        (double)L.g.V * (fine_link_cx(L) * lb + vb));
  int rc = wilson_soa_fused(L.g, fine_lcode(L, lp), fine_links(L, lp), prec, L.m, in, out, nrhs, bsub, reduce ? c->dred : nullptr,
                            red_dst ? red_dst : c->red_out, 4, c->st, out32);
  prof_end(c, slot);
  return rc;
}

// ------------------------------------------------------------ MR smoother
// Fine-level smoother of the mixed-precision cycle with the MR residuals
// s_k and q_k = A s_k stored in FP16 (FP16 links; the hopping sums of the
// MR steps in packed FP16 arithmetic, everything else FP32).  The
// cycle input r is used as r/|r| (|r|^2 per rhs in rn2, stride 4): the cycle
// is homogeneous in r, the restricted residual was scaled the same way, so
// e here belongs to r/|r| and every stored residual is O(1).
static int mr_smooth_h16(wmg_ctx *c, const void *r, const double *rn2, void *e, int nsteps, int nrhs) {
  Level &L = c->lv[0];
  void *sv[4] = {nullptr, nullptr, nullptr, nullptr}, *q;
  const int names[4] = {VS, VS1, VS2, VS3};
  if (L.n % 4) return set_error(-1, "mr_smooth_h16: length %ld not a multiple of 4", L.n);
  for (int k = 0; k < nsteps; k++) TRY(level_vec(c, 0, P16, names[k], &sv[k], nrhs));
  TRY(level_vec(c, 0, P16, VQ, &q, nrhs));
  const double vb = (double)L.g.V * fine_link_cx(L) * 4;  // FP16 links
  c->st_fine++;
  int slot = prof_begin(c, K_DSLASH_RES, vb + (double)L.g.V * 12 * (8 + 8 + 4) * nrhs);
  int rc = wilson_soa_h16(L.g, fine_links(L, P16), P32, L.m, e, sv[0], nrhs, r, rn2, 4, nullptr, nullptr, 0, c->st,
                          L.lk);
  prof_end(c, slot);
  TRY(rc);
  dim3 g = grid_for<__half2>(L.n, nrhs);
  for (int k = 0; k < nsteps; k++) {
    c->st_fine++;
    slot = prof_begin(c, K_DSLASH_CYCLE, vb + (double)L.g.V * 12 * (4 + 4) * nrhs);
    rc = wilson_soa_h16(L.g, fine_links(L, P16), P16, L.m, sv[k], q, nrhs, nullptr, nullptr, 0, c->dred,
                        c->mr_red + (size_t)k * 64 * 4, 4, c->st, L.lk);
    prof_end(c, slot);
    TRY(rc);
    if (k + 1 < nsteps) {
      hipLaunchKernelGGL(k_mr_next<__half2>, g, dim3(256), 0, c->st, c->mr_red, k, (const __half2 *)sv[k],
                         (const __half2 *)q, (__half2 *)sv[k + 1], L.n);
      WMG_HIP(hipGetLastError());
    }
  }
  MrVecs mv{{sv[0], sv[1], sv[2], sv[3]}};
  hipLaunchKernelGGL((k_mr_accum<float2, __half2>), g, dim3(256), 0, c->st, c->mr_red, nsteps, mv, (float2 *)e, L.n);
  WMG_HIP(hipGetLastError());
  return 0;
}

// nsteps minimal-residual steps on A e = r from e (post-smoother, Sec. 3).
// On the fine level the residual and the two step reductions are fused into
// the operator's kernel.
// ------------------------------------------------------------ red/black smoother
// Red/black form of the fine-level post-smoother (Sec. 3, MG combined with
// red/black preconditioning): with s = r - D e, the correction d of D d = s
// has d_e from nsteps MR steps on the Schur complement
//   S d_e = s_e - D_eo D_oo^-1 s_o,  S = (4+m) - D_eo D_oe / (4+m)
// (from d_e = 0, solution update deferred as in mr_smooth), and
// d_o = D_oo^-1 (s_o - D_oe d_e); then e += d.  With D_{p,1-p} = -H_p/2:
// S x = (4+m) x - H_e(H_o(x)) / (4 (4+m)), the right-hand side is
// s_e + H_e(s_o) / (2 (4+m)) and d_o = (s_o + H_o(d_e) / 2) / (4+m).
static int eo_links(wmg_ctx *c, int lp, const void **Ue) {
  Level &F = c->lv[0];
  if (!F.Ue[lp]) {
    const size_t cs[3] = {16, 8, 4};
    TRY(dalloc(&F.Ue[lp], cs[lp] * 2 * 4 * (F.lk ? 6 : 9) * (size_t)eo_stride(F.g)));
    TRY(links_to_eo(F.g, F.U[P64], lp | F.lk, F.Ue[lp], c->st));
  }
  *Ue = F.Ue[lp];
  return 0;
}

// prec P64: all in FP64.  prec P16: r FP32 used as r/|r| (|r|^2 in rn2),
// sublattice vectors, MR iterates and the even correction d_e FP16, e FP32.
// e16 (prec P16 only): the prolonged correction in FP16 as the residual's
// input and the base of the last step, which then writes e = e16 + d
// without reading e.
static int mr_smooth_eo(wmg_ctx *c, int sp, const void *r, const double *rn2, void *e, int nsteps, int nrhs,
                        const void *e16 = nullptr, int ep = P32) {
  Level &L = c->lv[0];
  const int lp = sp == P64 ? P64 : P16;   // link precision
  const int vp = sp == P64 ? P64 : P16;   // sublattice residuals and MR iterates
  const int dp = sp == P64 ? P64 : P16;   // even correction d_e
  const void *Ue;
  TRY(eo_links(c, lp, &Ue));
  const int lc = lp | L.lk;
  void *s = nullptr, *xk[4] = {nullptr, nullptr, nullptr, nullptr}, *q, *t, *se, *so, *de;
  const int names[4] = {VH0, VH1, VH2, VH3};
  if (sp == P64) TRY(level_vec(c, 0, vp, VS, &s, nrhs));
  for (int k = 0; k < nsteps; k++) TRY(level_vec(c, 0, vp, names[k], &xk[k], nrhs));
  TRY(level_vec(c, 0, vp, VHQ, &q, nrhs));
  TRY(level_vec(c, 0, vp, VHT, &t, nrhs));
  TRY(level_vec(c, 0, vp, VHSE, &se, nrhs));
  TRY(level_vec(c, 0, vp, VHSO, &so, nrhs));
  TRY(level_vec(c, 0, dp, VHDE, &de, nrhs));
  const double m4 = 4.0 + L.m;
  const long nh = 12 * eo_stride(L.g);
  const double vb = (double)L.g.V * fine_link_cx(L) * (lp == P64 ? 16 : 4);  // links of both halves
  const double eb = sp == P64 ? 16 : 4;                                        // sublattice element bytes
  const double db = sp == P64 ? 16 : 4;                                        // d_e element bytes
  const double fb = sp == P64 ? 16 : (ep == P16 ? 4 : 8);                      // e element bytes
  const double hs = (double)L.g.V / 2 * 12 * nrhs;                             // elements of one half field
  // one red/black hop launch, timed and counted as the cycle's fine operator
  // (algorithmic bytes: the links of both halves, the input, the output and
  // the diagonal input when there is one)
  auto hop = [&](int par, double a, double b, int pdg, const void *dg, int phop, const void *in, int pout, void *out,
                 double *red, double *red_out, double bytes) -> int {
    const int slot = prof_begin(c, sp == P64 ? K_DSLASH_64 : K_DSLASH_CYCLE, bytes);
    const int rc = hop_eo(L.g, lc, Ue, par, a, b, pdg, dg, phop, in, pout, out, nrhs, red, red_out, 4, c->st);
    prof_end(c, slot);
    return rc;
  };
  // s = r - D e (full lattice; FP16 on the normalised problem), split
  c->st_fine++;
  int slot;
  if (sp == P64) {
    TRY(fine_apply_fused(c, P64, e, s, nrhs, r, false));
  } else {
    // written straight into the two half-lattice arrays
    slot = prof_begin(c, K_DSLASH_RES, vb + (double)L.g.V * 12 * ((e16 ? 4 : 8) + 8 + 4) * nrhs);
    int rc = wilson_soa_h16(L.g, fine_links(L, P16), e16 ? P16 : P32, L.m, e16 ? e16 : e, se, nrhs, r, rn2, 4,
                            nullptr, nullptr, 0, c->st, L.lk, so);
    prof_end(c, slot);
    TRY(rc);
  }
  if (sp == P64) TRY(eo_pack(L.g, vp, s, vp, se, so, nrhs, c->st));
  // x_0 = s_e + H_e(s_o) / (2 (4+m))
  TRY(hop(0, 1.0, 0.5 / m4, vp, se, vp, so, vp, xk[0], nullptr, nullptr, vb + 3 * hs * eb));
  dim3 g = sp == P64 ? grid_for<double2>(nh, nrhs) : grid_for<__half2>(nh, nrhs);
  for (int k = 0; k < nsteps; k++) {
    // q = S x_k with <q, x_k>, |q|^2 -> mr_red[k]; x_{k+1} = x_k - alpha_k q
    c->st_fine++;
    TRY(hop(1, 0.0, 1.0, vp, nullptr, vp, xk[k], vp, t, nullptr, nullptr, vb + 2 * hs * eb));
    TRY(hop(0, m4, -0.25 / m4, vp, xk[k], vp, t, vp, q, c->dred, c->mr_red + (size_t)k * 64 * 4,
            vb + 3 * hs * eb));
    if (k + 1 < nsteps) {
      if (sp == P64)
        hipLaunchKernelGGL(k_mr_next<double2>, g, dim3(256), 0, c->st, c->mr_red, k, (const double2 *)xk[k],
                           (const double2 *)q, (double2 *)xk[k + 1], nh);
      else
        hipLaunchKernelGGL(k_mr_next<__half2>, g, dim3(256), 0, c->st, c->mr_red, k, (const __half2 *)xk[k],
                           (const __half2 *)q, (__half2 *)xk[k + 1], nh);
      WMG_HIP(hipGetLastError());
    }
  }
  // d_e = sum_k alpha_k x_k
  MrVecs mv{{xk[0], xk[1], xk[2], xk[3]}};
  if (sp == P64)
    hipLaunchKernelGGL((k_mr_accum<double2, double2, 0>), g, dim3(256), 0, c->st, c->mr_red, nsteps, mv,
                       (double2 *)de, nh);
  else
    hipLaunchKernelGGL((k_mr_accum<__half2, __half2, 0>), g, dim3(256), 0, c->st, c->mr_red, nsteps, mv,
                       (__half2 *)de, nh);
  WMG_HIP(hipGetLastError());
  // d_o = (s_o + H_o(d_e) / 2) / (4+m) and e += (d_e, d_o) in one kernel
  // (bytes: links, s_o, d_e, and e read and written; with e16 the FP16 base
  // read and e written)
  const int slot2 = prof_begin(c, sp == P64 ? K_DSLASH_64 : K_DSLASH_CYCLE,
                               vb + hs * (eb + db + (e16 ? 2 * 4 + 2 * fb : 4 * fb)));
  const int rc2 = hop_eo_add(L.g, lc, Ue, 1.0 / m4, 0.5 / m4, vp, so, dp, de, e, nrhs, c->st, e16,
                             sp == P64 ? P64 : ep);
  prof_end(c, slot2);
  return rc2;
}

static int mr_smooth(wmg_ctx *c, int l, int prec, const void *r, void *e, int nsteps, int nrhs,
                     bool in_cycle = false) {
  Level &L = c->lv[l];
  if (in_cycle && L.fine && prec == P64 && (c->p.flags & WMG_EO_SMOOTHER) && nsteps >= 1 && nsteps <= 4 && nrhs <= 64)
    return mr_smooth_eo(c, P64, r, nullptr, e, nsteps, nrhs);
  void *s, *q;
  TRY(level_vec(c, l, prec, VS, &s, nrhs));
  TRY(level_vec(c, l, prec, VQ, &q, nrhs));
  if (L.fine && nsteps >= 1 && nsteps <= 4 && nrhs <= 64) {
    // s_0 = r - A e; q_k = A s_k with <q_k,s_k>, |q_k|^2 fused;
    // s_{k+1} = s_k - alpha_k q_k; finally e += sum_k alpha_k s_k
    void *sv[4] = {s, nullptr, nullptr, nullptr};
    const int names[4] = {VS, VS1, VS2, VS3};
    for (int k = 1; k < nsteps; k++) TRY(level_vec(c, l, prec, names[k], &sv[k], nrhs));
    TRY(fine_apply_fused(c, prec, e, s, nrhs, r, false));
    dim3 g = prec == P64 ? grid_for<double2>(L.n, nrhs) : grid_for<float2>(L.n, nrhs);
    for (int k = 0; k < nsteps; k++) {
      TRY(fine_apply_fused(c, prec, sv[k], q, nrhs, nullptr, true, c->mr_red + (size_t)k * 64 * 4));
      if (k + 1 < nsteps) {
        if (prec == P64)
          hipLaunchKernelGGL(k_mr_next<double2>, g, dim3(256), 0, c->st, c->mr_red, k, (const double2 *)sv[k],
                             (const double2 *)q, (double2 *)sv[k + 1], L.n);
        else
          hipLaunchKernelGGL(k_mr_next<float2>, g, dim3(256), 0, c->st, c->mr_red, k, (const float2 *)sv[k],
                             (const float2 *)q, (float2 *)sv[k + 1], L.n);
        WMG_HIP(hipGetLastError());
      }
    }
    MrVecs mv{{sv[0], sv[1], sv[2], sv[3]}};
    if (prec == P64)
      hipLaunchKernelGGL(k_mr_accum<double2>, g, dim3(256), 0, c->st, c->mr_red, nsteps, mv, (double2 *)e, L.n);
    else
      hipLaunchKernelGGL(k_mr_accum<float2>, g, dim3(256), 0, c->st, c->mr_red, nsteps, mv, (float2 *)e, L.n);
    WMG_HIP(hipGetLastError());
    return 0;
  }
  if (L.fine) {
    TRY(fine_apply_fused(c, prec, e, s, nrhs, r, false));
  } else {
    TRY(apply_op(c, l, prec, e, q, nrhs, true));
    TRY(csub(prec, r, q, s, L.n, nrhs, c->st));
  }
  for (int k = 0; k < nsteps; k++) {
    if (L.fine) {
      TRY(fine_apply_fused(c, prec, s, q, nrhs, nullptr, true));
    } else {
      TRY(apply_op(c, l, prec, s, q, nrhs, true));
      TRY(dot_norm(c->red, prec, q, s, L.n, nrhs, c->red_out, 4, c->st));
    }
    dim3 g = grid_for<double2>(L.n, nrhs);
    if (prec == P64)
      hipLaunchKernelGGL(k_mr_update<double2>, g, dim3(256), 0, c->st, c->red_out, (double2 *)e, (double2 *)s,
                         (const double2 *)q, L.n);
    else
      hipLaunchKernelGGL(k_mr_update<float2>, g, dim3(256), 0, c->st, c->red_out, (float2 *)e, (float2 *)s,
                         (const float2 *)q, L.n);
    WMG_HIP(hipGetLastError());
  }
  return 0;
}

// ------------------------------------------------------------ CGNR
// CG on the normal equations at the coarsest level (Sec. 3); stops per rhs
// when |b - A x| <= tol |b| (recursively updated residual).
static int cgnr(wmg_ctx *c, int l, int prec, const void *b, void *x, int nrhs) {
  Level &L = c->lv[l];
  void *r, *s, *p, *u;
  TRY(level_vec(c, l, prec, VCR, &r, nrhs));
  TRY(level_vec(c, l, prec, VCS, &s, nrhs));
  TRY(level_vec(c, l, prec, VCP, &p, nrhs));
  TRY(level_vec(c, l, prec, VCU, &u, nrhs));
  double tol = c->p.coarse_tol;
  TRY(zero(prec, x, L.n, nrhs, c->st));
  TRY(copy(prec, r, prec, b, L.n, nrhs, c->st));
  // cg[rhs*8 + 4] = |b|^2
  TRY(norm2(c->red, prec, b, L.n, nrhs, c->cg + 4, 8, c->st));
  hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(64), 0, c->st, c->cg, nrhs, tol * tol, (const double *)nullptr);
  TRY(apply_op(c, l, prec, r, s, nrhs, false, 1, c->cg + 1, 8));
  TRY(copy(prec, p, prec, s, L.n, nrhs, c->st));
  int cur = 1;
  constexpr int check = 4;
  int it = 0;
  dim3 g = grid_for<double2>(L.n, nrhs);
  double *spart;
  TRY(cpart_get(c, (size_t)nrhs * (g.x > L.g.V ? g.x : L.g.V), &spart));
  // first half of iteration it (slot cur): u = A p, |u|^2; x += alpha p,
  // r -= alpha u, |r|^2; convergence flag
  auto half1 = [&](int cu) -> int {
    TRY(apply_op(c, l, prec, p, u, nrhs, false, 0, c->cg + 0, 8));
    if (prec == P64)
      hipLaunchKernelGGL(k_cg_step1<double2>, g, dim3(256), 0, c->st, c->cg, cu, (double2 *)x, (double2 *)r,
                         (const double2 *)p, (const double2 *)u, L.n, nrhs, spart);
    else
      hipLaunchKernelGGL(k_cg_step1<float2>, g, dim3(256), 0, c->st, c->cg, cu, (float2 *)x, (float2 *)r,
                         (const float2 *)p, (const float2 *)u, L.n, nrhs, spart);
    TRY(sum_partials(spart, g.x, nrhs, c->cg + 3, 8, c->st));
    hipLaunchKernelGGL(k_cg_check, dim3(1), dim3(64), 0, c->st, c->cg, nrhs, c->flag);
    WMG_HIP(hipGetLastError());
    return 0;
  };
  // second half: s = A^dag r, |s|^2 (slot nxt); p = s + beta p
  auto half2 = [&](int cu) -> int {
    const int nxt = 3 - cu;
    TRY(apply_op(c, l, prec, r, s, nrhs, false, 1, c->cg + nxt, 8));
    if (prec == P64)
      hipLaunchKernelGGL(k_cg_step2<double2>, g, dim3(256), 0, c->st, c->cg, nxt, cu, (const double2 *)s,
                         (double2 *)p, L.n);
    else
      hipLaunchKernelGGL(k_cg_step2<float2>, g, dim3(256), 0, c->st, c->cg, nxt, cu, (const float2 *)s,
                         (float2 *)p, L.n);
    WMG_HIP(hipGetLastError());
    return 0;
  };
  // With WMG_GRAPHS the loop runs as HIP graphs of `check` iterations (the
  // same launches in the same order, so the same results): the graph of a
  // buffer set is captured the second time the set is used (the first run
  // fills every lazily allocated buffer and tuner choice), then replayed.
  wmg_ctx::CgGraph *G = nullptr;
  if ((c->p.flags & WMG_GRAPHS) && !c->prof && c->p.coarse_maxiter % check == 0) {
    std::vector<uintptr_t> key = {(uintptr_t)l, (uintptr_t)prec, (uintptr_t)nrhs, (uintptr_t)x, (uintptr_t)r,
                                  (uintptr_t)s, (uintptr_t)p, (uintptr_t)u, (uintptr_t)spart, (uintptr_t)L.n};
    G = &c->cg_graphs[key];
    if (G->failed) G = nullptr;
    else if (!G->blk && G->seen++ >= 1) {
      auto capture = [&](auto body, hipGraphExec_t *out) -> int {
        hipGraph_t graph = nullptr;
        WMG_HIP(hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal));
        int rc = body();
        hipError_t e = hipStreamEndCapture(c->st, &graph);
        if (rc || e != hipSuccess || !graph) {
          if (graph) (void)hipGraphDestroy(graph);
          return rc ? rc : set_error(WMG_EHIP, "graph capture failed");
        }
        e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        return e == hipSuccess ? 0 : set_error(WMG_EHIP, "graph instantiation failed");
      };
      int rc = capture([&]() -> int {
        int cu = 1;
        for (int k = 0; k < check; k++) {
          TRY(half1(cu));
          if (k + 1 < check) {
            TRY(half2(cu));
            cu = 3 - cu;
          }
        }
        return 0;
      }, &G->blk);
      // the last iteration of a block has slot 1 when check is odd, else 2
      if (!rc) rc = capture([&]() -> int { return half2(((check - 1) % 2) ? 2 : 1); }, &G->tail);
      if (rc) {
        (void)hipGetLastError();
        G->failed = true;
        G = nullptr;
      }
    } else if (!G->blk) {
      G = nullptr;
    }
  }
  if (G) {
    // blocks of `check` iterations; the block ends after the first half of
    // its last iteration, where the flag is read (an even `check` brings
    // every block back to slot 1)
    static_assert(check % 2 == 0, "blocks of an even iteration count start in slot 1");
    for (; it < c->p.coarse_maxiter; it += check) {
      WMG_HIP(hipGraphLaunch(G->blk, c->st));
      int done = 0;
      WMG_HIP(hipMemcpyAsync(&done, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->st));
      TRY(sync(c));
      if (done) {
        it += check;
        break;
      }
      if (it + check < c->p.coarse_maxiter) WMG_HIP(hipGraphLaunch(G->tail, c->st));
    }
  } else {
    for (; it < c->p.coarse_maxiter; it++) {
      TRY(half1(cur));
      if ((it + 1) % check == 0 || it + 1 == c->p.coarse_maxiter) {
        int done = 0;
        WMG_HIP(hipMemcpyAsync(&done, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->st));
        TRY(sync(c));
        if (done) { it++; break; }
      }
      TRY(half2(cur));
      cur = 3 - cur;
    }
  }
  // effective iterations (max over rhs) for the statistics
  WMG_HIP(hipMemcpyAsync(c->hbuf, c->cg, sizeof(double) * 8 * nrhs, hipMemcpyDeviceToHost, c->st));
  TRY(sync(c));
  double mx = 0;
  for (int r2 = 0; r2 < nrhs; r2++) mx = fmax(mx, c->hbuf[r2 * 8 + 6]);
  c->st_coarse += (long)mx;
  return 0;
}

// ------------------------------------------------------------ cycle
// e = M_l r: restrict, coarse correction (CGNR at the coarsest level, else
// one or two recursive cycles), prolong, post-smooth (no pre-smoothing).
// rn2: |r|^2 per rhs (device, stride 4) when the caller already has it
// The fine-level cycle of a mixed solve can write its output e in FP16
// (e16out): with the red/black smoother, FP16 prolongation, 1-4 MR steps,
// at most 64 rhs, unless WMG_Z32.
static bool z16_ok(wmg_ctx *c, int l, int prec, int nrhs) {
  return l == 0 && prec == P32 && c->lv[0].fine && c->nl_cur > 1 && c->p.post_smooth >= 1 &&
         c->p.post_smooth <= 4 && nrhs <= 64 && (c->p.flags & WMG_EO_SMOOTHER) && !(c->p.flags & WMG_Z32) &&
         prolong16_ok(c, 0, nrhs);
}

static int mg_cycle_l(wmg_ctx *c, int l, int prec, const void *r, void *e, int nrhs, const double *rn2 = nullptr,
                      bool e16out = false) {
  if (e16out && !z16_ok(c, l, prec, nrhs)) return set_error(-1, "mg_cycle: FP16 output not available here");
  Level &C = c->lv[l + 1];
  void *rc, *ec;
  TRY(level_vec(c, l + 1, prec, VR, &rc, nrhs));
  TRY(level_vec(c, l + 1, prec, VE, &ec, nrhs));
  // FP32 cycle on the fine level: FP16 smoother storage on the normalised
  // problem r/|r| (e comes out scaled by 1/|r|, which the flexible outer
  // solver absorbs)
  const bool h16 = l == 0 && prec == P32 && c->lv[0].fine && c->p.post_smooth >= 1 && c->p.post_smooth <= 4 &&
                   nrhs <= 64;
  if (h16) {
    if (rn2)
      WMG_HIP(hipMemcpyAsync(c->cyc_nrm, rn2, sizeof(double) * (4 * (size_t)(nrhs - 1) + 1), hipMemcpyDeviceToDevice,
                             c->st));
    else
      TRY(norm2(c->red, P32, r, c->lv[0].n, nrhs, c->cyc_nrm, 4, c->st));
  }
  TRY(transfer_restrict(c, l, prec, r, rc, nrhs, h16 ? c->cyc_nrm : nullptr));
  if (h16) TRY(scale_inv_sqrt(P32, rc, c->cyc_nrm, 4, C.n, nrhs, c->st));
  if (l + 1 == c->nl_cur - 1) {
    TRY(cgnr(c, l + 1, prec, rc, ec, nrhs));
  } else {
    TRY(mg_cycle_l(c, l + 1, prec, rc, ec, nrhs));
    if (c->p.cycle == WMG_WCYCLE) {
      void *t, *e2;
      TRY(level_vec(c, l + 1, prec, VT, &t, nrhs));
      TRY(level_vec(c, l + 1, prec, VE2, &e2, nrhs));
      TRY(apply_op(c, l + 1, prec, ec, t, nrhs, true));
      TRY(csub(prec, rc, t, t, C.n, nrhs, c->st));
      TRY(mg_cycle_l(c, l + 1, prec, t, e2, nrhs));
      TRY(axpby(prec, 1.0, e2, 1.0, ec, C.n, nrhs, c->st));  // ec += e2
    }
  }
  if (h16 && (c->p.flags & WMG_EO_SMOOTHER) && prolong16_ok(c, l, nrhs)) {
    // the red/black smoother reads the prolonged correction in FP16 and
    // writes e = P ec + d
    void *eh;
    TRY(level_vec(c, 0, P16, VEH, &eh, nrhs));
    TRY(transfer_prolong(c, l, prec, ec, eh, nrhs, true));
    return mr_smooth_eo(c, P16, r, c->cyc_nrm, e, c->p.post_smooth, nrhs, eh, e16out ? P16 : P32);
  }
  TRY(transfer_prolong(c, l, prec, ec, e, nrhs));
  if (h16 && (c->p.flags & WMG_EO_SMOOTHER)) return mr_smooth_eo(c, P16, r, c->cyc_nrm, e, c->p.post_smooth, nrhs);
  if (h16) return mr_smooth_h16(c, r, c->cyc_nrm, e, c->p.post_smooth, nrhs);
  TRY(mr_smooth(c, l, prec, r, e, c->p.post_smooth, nrhs, true));
  return 0;
}

// ------------------------------------------------------------ GCR buffers
static int gcr_buffers(wmg_ctx *c, int l, int prec, int nrhs, GcrBuf **out) {
  int slot = (l == 0 ? 0 : 1);
  GcrBuf &B = c->gb[slot][prec == P64 ? 0 : 1];
  Level &L = c->lv[l];
  long nalloc = L.n_alloc;
  bool ok = B.x64 && B.prec == prec && B.nrhs >= nrhs && B.n >= nalloc;
  if (!ok) {
    // release and reallocate
    for (int k = 0; k < KMAX; k++) {
      if (B.z[k]) (void)hipFree(B.z[k]);
      if (B.wv[k]) (void)hipFree(B.wv[k]);
      B.z[k] = B.wv[k] = nullptr;
    }
    if (B.x64) (void)hipFree(B.x64);
    if (B.r64) (void)hipFree(B.r64);
    if (B.b64) (void)hipFree(B.b64);
    if (B.t64) (void)hipFree(B.t64);
    if (B.prec != P64 && B.rin) (void)hipFree(B.rin);
    if (B.zdev) (void)hipFree(B.zdev);
    if (B.wdev) (void)hipFree(B.wdev);
    B = GcrBuf();
    B.prec = prec;
    B.nrhs = nrhs;
    B.n = nalloc;
    int K = c->p.gcr_restart;
    for (int k = 0; k < K; k++) {
      TRY(dalloc(&B.z[k], csize(prec) * nalloc * nrhs));
      TRY(dalloc(&B.wv[k], csize(prec) * nalloc * nrhs));
    }
    TRY(dalloc((void **)&B.x64, 16 * nalloc * nrhs));
    TRY(dalloc((void **)&B.r64, 16 * nalloc * nrhs));
    TRY(dalloc((void **)&B.b64, 16 * nalloc * nrhs));
    TRY(dalloc((void **)&B.t64, 16 * nalloc * nrhs));
    if (prec == P64) B.rin = B.r64;
    else TRY(dalloc(&B.rin, csize(prec) * nalloc * nrhs));
    TRY(dalloc((void **)&B.zdev, sizeof(void *) * KMAX));
    TRY(dalloc((void **)&B.wdev, sizeof(void *) * KMAX));
    // on the context's stream, ahead of the kernels that read the tables
    WMG_HIP(hipMemcpyAsync(B.zdev, B.z, sizeof(void *) * KMAX, hipMemcpyHostToDevice, c->st));
    WMG_HIP(hipMemcpyAsync(B.wdev, B.wv, sizeof(void *) * KMAX, hipMemcpyHostToDevice, c->st));
    WMG_HIP(hipStreamSynchronize(c->st));
  }
  *out = &B;
  return 0;
}

// ------------------------------------------------------------ flexible GCR
// Restarted flexible GCR on level l (Sec. 3 outer solver) with reliable
// updates.  Each restart cycle works in the inner precision on r_in: z_k =
// M(r_in), w_k = A z_k orthonormalised against w_0..w_{k-1} (classical GS
// twice), alpha_k = <w_k, r_in>, r_in -= alpha_k w_k.  A right-hand side
// leaves the cycle when |r_in| <= tol |b|, when |r_in| < delta |r| (mixed
// precision) or after K steps; the FP64 solution update is recovered from
// the triangular system A z_k = gamma_k w_k + sum_j beta_jk w_j, and the
// residual is recomputed in FP64 (the reliable update).
// precond: 0 = smoother only (first setup vector), 1 = multigrid cycle.
// r = b - A x in FP64 and |r|^2 per rhs into c->red_out[rhs*4 + *off]; on
// the fine level one fused operator launch (residual and norm in its
// epilogue), elsewhere operator, subtraction and norm.
// r = b - A x in FP64 and |r|^2 (at red_out[4 rhs + *off]); on the fine level
// of a mixed solve the kernel writes r only as the FP32 copy in B.rin
// (*rin_done = true), which is all the inner cycle reads, and the norm from
// the FP64 values
static int residual64(wmg_ctx *c, int l, GcrBuf &B, int nrhs, int *off, bool *rin_done) {
  Level &L = c->lv[l];
  *rin_done = false;
  if (L.fine) {
    *off = 2;
    *rin_done = B.prec == P32;
    return B.prec == P32 ? fine_apply_fused(c, P64, B.x64, nullptr, nrhs, B.b64, true, nullptr, B.rin)
                         : fine_apply_fused(c, P64, B.x64, B.r64, nrhs, B.b64, true);
  }
  *off = 0;
  TRY(apply_op(c, l, P64, B.x64, B.t64, nrhs, false));
  TRY(csub(P64, B.b64, B.t64, B.r64, L.n, nrhs, c->st));
  return norm2(c->red, P64, B.r64, L.n, nrhs, c->red_out, 4, c->st);
}

// w = A z on the fine level from the FP16-stored preconditioner output z:
// FP32 links and arithmetic, FP32 w; with r (FP32) also <w, r> and |w|^2
// per rhs into c->red_out[4 rhs + 0..2] (the first step of a restart)
static int apply_outer_z16(wmg_ctx *c, const void *z, void *w, int nrhs, const void *r = nullptr) {
  Level &L = c->lv[0];
  c->st_fine++;
  const double vb = (12.0 * 4 + 12.0 * 8 + (r ? 12.0 * 8 : 0.0)) * nrhs;  // z, w and r
  const int slot = prof_begin(c, K_DSLASH_OUTER32, (double)L.g.V * (fine_link_cx(L) * 8 + vb));
  const int rc = wilson_soa_in16(L.g, fine_lcode(L, P32), fine_links(L, P32), L.m, z, w, nrhs, c->st,
                                 r ? c->dred : nullptr, r ? c->red_out : nullptr, 4, r);
  prof_end(c, slot);
  return rc;
}

static int gcr_solve(wmg_ctx *c, int l, GcrBuf &B, int nrhs, double tol, int maxiter, int precond, double delta,
                     bool x0_nonzero, std::vector<int> &iters, double *relres_out) {
  Level &L = c->lv[l];
  const int ip = B.prec;
  // The flexible GCR takes any preconditioner output: where the cycle can
  // write z in FP16, z is stored so, and A z and the solution update read the
  // same FP16 values (z is the cycle's output for r/|r|, O(1)).
  const int zp = precond == 1 && z16_ok(c, l, ip, nrhs) ? P16 : ip;
  const int K = c->p.gcr_restart;
  const long n = L.n;
  hipStream_t st = c->st;
  if (B.zfmt >= 0 && B.zfmt != zp)
    for (int k = 0; k < K; k++) TRY(zero(ip, B.z[k], n, B.nrhs, st));
  B.zfmt = zp;
  std::vector<double> bn(nrhs), rn(nrhs), rn_last(nrhs);
  std::vector<char> active(nrhs), frozen(nrhs);
  iters.assign(nrhs, 0);
  // |b|
  TRY(norm2(c->red, P64, B.b64, n, nrhs, c->red_out, 4, st));
  WMG_HIP(hipMemcpyAsync(c->hbuf, c->red_out, sizeof(double) * 4 * nrhs, hipMemcpyDeviceToHost, st));
  TRY(sync(c));
  for (int r = 0; r < nrhs; r++) bn[r] = sqrt(c->hbuf[4 * r]);
  int roff = 0;
  bool rin_done = false;  // B.rin already holds the FP32 copy of r
  // without an initial guess x is zero but not yet written: the first
  // solution update writes it instead of adding to it
  bool x_unset = !x0_nonzero;
  if (x0_nonzero) {
    TRY(residual64(c, l, B, nrhs, &roff, &rin_done));
  } else if (ip != P64) {
    // r = b: the first inner cycle starts from the FP32 copy of b, |r|^2 =
    // |b|^2 is already in red_out, and r64 is first written by the reliable
    // update
    TRY(copy(ip, B.rin, P64, B.b64, n, nrhs, st));
    rin_done = true;
  } else {
    TRY(copy(P64, B.r64, P64, B.b64, n, nrhs, st));
    TRY(norm2(c->red, P64, B.r64, n, nrhs, c->red_out, 4, st));
  }
  WMG_HIP(hipMemcpyAsync(c->hbuf, c->red_out, sizeof(double) * 4 * nrhs, hipMemcpyDeviceToHost, st));
  TRY(sync(c));
  bool any = false;
  for (int r = 0; r < nrhs; r++) {
    rn[r] = sqrt(c->hbuf[4 * r + roff]);
    active[r] = !(rn[r] <= tol * bn[r]);
    if (!std::isfinite(rn[r])) return set_error(WMG_EBREAKDOWN, "non-finite initial residual");
    any |= active[r];
  }
  int total = 0;
  std::vector<double> mask(nrhs * GS, 0.0);
  while (any && total < maxiter) {
    for (int r = 0; r < nrhs; r++) {
      rn_last[r] = rn[r];
      frozen[r] = !active[r];
    }
    if (ip != P64 && !rin_done) TRY(copy(ip, B.rin, P64, B.r64, n, nrhs, st));
    int k = 0;
    while (k < K && total < maxiter) {
      // per-rhs participation mask of this step
      double *hm = c->hbuf + 2048;
      for (int r = 0; r < nrhs; r++) hm[r] = frozen[r] ? 0.0 : 1.0;
      WMG_HIP(hipMemcpyAsync(c->mask, hm, sizeof(double) * nrhs, hipMemcpyHostToDevice, st));
      void *z = B.z[k], *w = B.wv[k];
      if (precond == 1) {
        // |r_in|^2 is at hand: from the last reliable update (k = 0) or
        // from the previous step's r_in update
        TRY(mg_cycle_l(c, l, ip, B.rin, z, nrhs, c->red_out + (k == 0 ? roff : 0), zp == P16));
      } else {
        TRY(zero(ip, z, n, nrhs, st));
        TRY(mr_smooth(c, l, ip, B.rin, z, c->p.post_smooth, nrhs));
      }
      // the first step's <w, r> and |w|^2 come from the operator's epilogue
      // when z is FP16
      if (zp == P16) TRY(apply_outer_z16(c, z, w, nrhs, k == 0 ? B.rin : nullptr));
      else TRY(apply_op(c, l, ip, z, w, nrhs, false));
      // classical Gram-Schmidt against the unnormalised w_j, fused: dots |
      // project + <w, r> + |w|^2 (FP64: dots | project + new dots | project
      // + <w, r> + |w|^2)
      if (k == 0) {
        if (zp != P16) TRY(dot_norm(c->red, ip, w, B.rin, n, nrhs, c->red_out, 4, st));
      } else {
        TRY(multi_dot(c->red, ip, (const void *const *)B.wdev, k, w, n, nrhs, c->gcr + G_TMP, GS, st));
        // FP32 inner solve: one projection pass (on the 32^3x64, 28-rhs
        // mixed solve the outer, coarse and reliable-update counts are those
        // of two passes, and the solve is 3 % faster); FP64: two passes
        if (ip != P64) {
          TRY(gcr_project(c->red, ip, 3, (const void *const *)B.wdev, k, w, B.rin, c->gcr + G_TMP, GS,
                          c->gcr + G_GAMMA, GS, c->gcr + G_BETA, GS, k, n, nrhs, c->red_out, 4, st));
        } else {
          TRY(gcr_project(c->red, ip, 1, (const void *const *)B.wdev, k, w, nullptr, c->gcr + G_TMP, GS,
                          c->gcr + G_GAMMA, GS, c->gcr + G_BETA, GS, k, n, nrhs, c->gcr + G_TMP2, GS, st));
          TRY(gcr_project(c->red, ip, 2, (const void *const *)B.wdev, k, w, B.rin, c->gcr + G_TMP2, GS,
                          c->gcr + G_GAMMA, GS, c->gcr + G_BETA, GS, k, n, nrhs, c->red_out, 4, st));
        }
      }
      hipLaunchKernelGGL(k_gcr_alpha2, dim3(1), dim3(64), 0, st, c->gcr, c->red_out, c->mask, k, nrhs);
      // r_in -= alpha_k w_k and |r_in|^2
      TRY(caxpy_norm(c->red, ip, c->gcr + G_ALPHA + 2 * k, GS, w, B.rin, n, nrhs, c->red_out, 4, st));
      WMG_HIP(hipMemcpyAsync(c->hbuf, c->red_out, sizeof(double) * 4 * nrhs, hipMemcpyDeviceToHost, st));
      TRY(sync(c));
      bool allfrozen = true;
      for (int r = 0; r < nrhs; r++) {
        double rin = sqrt(c->hbuf[4 * r]);
        if (!std::isfinite(rin)) return set_error(WMG_EBREAKDOWN, "non-finite GCR residual (rhs %d)", r);
        if (!frozen[r]) {
          iters[r]++;
          if (rin <= tol * bn[r] || rin < delta * rn_last[r]) frozen[r] = 1;
        }
        allfrozen &= (bool)frozen[r];
      }
      k++;
      total++;
      if (allfrozen) break;
    }
    hipLaunchKernelGGL(k_gcr_trisolve2, dim3(1), dim3(64), 0, st, c->gcr, k, nrhs);
    TRY(multi_caxpy(P64, B.x64, zp, (const void *const *)B.zdev, k, c->gcr + G_C, GS, 1.0, x_unset ? 0 : 1, n,
                    nrhs, st));
    x_unset = false;
    // reliable update: true residual in FP64
    TRY(residual64(c, l, B, nrhs, &roff, &rin_done));
    c->st_rel++;
    WMG_HIP(hipMemcpyAsync(c->hbuf, c->red_out, sizeof(double) * 4 * nrhs, hipMemcpyDeviceToHost, st));
    TRY(sync(c));
    any = false;
    for (int r = 0; r < nrhs; r++) {
      rn[r] = sqrt(c->hbuf[4 * r + roff]);
      if (!std::isfinite(rn[r])) return set_error(WMG_EBREAKDOWN, "non-finite true residual (rhs %d)", r);
      if (active[r] && rn[r] <= tol * bn[r]) active[r] = 0;
      any |= (bool)active[r];
    }
  }
  if (x_unset) TRY(zero(P64, B.x64, n, nrhs, st));
  if (relres_out) {
    double mx = 0;
    for (int r = 0; r < nrhs; r++) mx = fmax(mx, bn[r] > 0 ? rn[r] / bn[r] : rn[r]);
    *relres_out = mx;
  }
  return any ? WMG_ENOTCONV : 0;
}

// ------------------------------------------------------------ hierarchy build
// P_l from the first k null vectors (Eq. 2.7, chirality split) and the
// Galerkin operator of level l+1.
static int build_level(wmg_ctx *c, int l, int k) {
  Level &F = c->lv[l], &C = c->lv[l + 1];
  F.nv = k;
  C.dof = F.ns * k;
  C.n = C.g.V * C.dof;
  WMG_HIP(hipMemsetAsync(c->flag, 0, sizeof(int), c->st));
  TRY(block_orthonormalize(F.g, F.dof, F.b, k, F.vecs, F.fine ? 1 : 0, F.P64, c->flag, c->st, F.ns));
  int fail = 0;
  WMG_HIP(hipMemcpyAsync(&fail, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->st));
  TRY(sync(c));
  if (fail) return set_error(WMG_ERANK, "block Gram-Schmidt breakdown at level %d (null vectors dependent)", l);
  TRY(coarse_build(F.g, F.fine ? 0 : 1, F.dof, F.U[P64], F.m, F.Y64, F.b, k, F.P64, C.Y64, nullptr, c->st, F.ns));
  return 0;
}

// The setup's rebuild after vector k-1 has been added: only that vector's
// block orthonormalisation and its columns (and, by gamma_5-hermiticity,
// rows) of the Galerkin operator are computed; the first k-1 stay as built
// (Ys holds the blocks with room for every vector of the level).
static int build_level_next(wmg_ctx *c, int l, int k, double2 *Ys) {
  Level &F = c->lv[l], &C = c->lv[l + 1];
  F.nv = k;
  C.dof = F.ns * k;
  C.n = C.g.V * C.dof;
  WMG_HIP(hipMemsetAsync(c->flag, 0, sizeof(int), c->st));
  TRY(block_orthonormalize(F.g, F.dof, F.b, k, F.vecs, F.fine ? 1 : 0, F.P64, c->flag, c->st, F.ns, k - 1));
  int fail = 0;
  WMG_HIP(hipMemcpyAsync(&fail, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->st));
  TRY(sync(c));
  if (fail) return set_error(WMG_ERANK, "block Gram-Schmidt breakdown at level %d (null vectors dependent)", l);
  TRY(coarse_build_next(F.g, F.fine ? 0 : 1, F.dof, F.U[P64], F.m, F.Y64, F.b, k, F.nv_max, F.P64, Ys, C.Y64, c->st,
                        F.ns));
  return 0;
}

// reduced-precision copies used by the mixed-precision cycle
static int make_low_precision(wmg_ctx *c) {
  if (c->p.precision != WMG_MIXED) return 0;
  for (int l = 0; l + 1 < c->nl; l++) {
    Level &F = c->lv[l];
    int bs = F.b[0] * F.b[1] * F.b[2] * F.b[3];
    long nsites = (long)F.nv * (F.g.V / bs) * bs;
    if (!F.P16) {
      TRY(dalloc((void **)&F.P16, 4 * (size_t)F.nv_max * F.g.V * F.dof));
      TRY(dalloc((void **)&F.Ps, 4 * (size_t)F.nv_max * F.g.V));
    }
    TRY(P_convert_half(nsites, bs, F.dof, F.fine ? 1 : 0, F.P64, F.P16, F.Ps, c->st));
  }
  for (int l = 1; l < c->nl; l++) {
    Level &C = c->lv[l];
    if (C.dof_max <= 64 && !(c->p.flags & WMG_COARSE_FP32)) {
      if (!C.Ymh) {
        TRY(dalloc((void **)&C.Ymh, sizeof(__half) * coarse_mfma_halfs(C.g.V, C.dof_max)));
        TRY(dalloc((void **)&C.Ymsc, sizeof(float) * 9 * (size_t)C.g.V));
      }
      if (!c->bpart) TRY(dalloc((void **)&c->bpart, sizeof(float) * COARSE_H_PART * COARSE_H_MAXRHS));
      TRY(coarse_to_mfma16(C.g.V, C.dof, C.Y64, C.Ymh, C.Ymsc, c->st));
    } else if (C.dof_max <= 64) {
      if (!C.Ym) TRY(dalloc((void **)&C.Ym, sizeof(float) * coarse_mfma_floats(C.g.V, C.dof_max)));
      TRY(coarse_to_mfma(C.g.V, C.dof, C.Y64, C.Ym, c->st));
    } else {
      long cnt = C.g.V * 9L * C.dof * C.dof;
      if (!C.Y32) TRY(dalloc((void **)&C.Y32, 8 * (size_t)C.g.V * 9 * C.dof_max * C.dof_max));
      TRY(coarse_convert(cnt, C.Y64, P32, C.Y32, c->st));
    }
  }
  return sync(c);
}

// Adaptive setup of level l (Sec. 2, Eq. 2.6): null vector k starts from a
// Philox random vector and is relaxed on A x = 0 by setup_iters GCR steps
// preconditioned with the trial two-level scheme built from vectors
// 0..k-1 (the smoother alone for k = 0); it is then normalised.  After the
// last vector the level is built from all of them.
static int setup_level(wmg_ctx *c, int l) {
  Level &F = c->lv[l];
  int nv = F.nv_max;
  c->nl_cur = l + 2;
  GcrBuf *B;
  TRY(gcr_buffers(c, l, P64, 1, &B));
  long n = F.n;
  std::vector<int> its;
  // blocks with room for every vector of the level, for the incremental
  // rebuilds (freed at the end of the level's setup)
  double2 *Ys = nullptr;
  {
    Level &C = c->lv[l + 1];
    const size_t nmax = (size_t)F.ns * nv;
    TRY(dalloc((void **)&Ys, sizeof(double2) * (size_t)C.g.V * 9 * nmax * nmax));
  }
  struct YsFree {
    double2 *p;
    ~YsFree() { if (p) (void)hipFree(p); }
  } ys_free{Ys};
  for (int k = 0; k < nv; k++) {
    TRY(start_vectors(F.g.V, F.dof, c->p.seed, l, k, 1, B->x64, F.fine ? 1 : 0, F.g.Vs, c->st));
    if (k > 0) TRY(build_level_next(c, l, k, Ys));
    TRY(zero(P64, B->b64, n, 1, c->st));
    int rc = gcr_solve(c, l, *B, 1, 0.0, c->p.setup_iters, k > 0 ? 1 : 0, 0.0, true, its, nullptr);
    if (rc < 0) return rc;
    TRY(norm2(c->red, P64, B->x64, n, 1, c->red_out, 4, c->st));
    TRY(scale_inv_sqrt(P64, B->x64, c->red_out, 4, n, 1, c->st));
    TRY(copy(P64, F.vecs + (size_t)k * n, P64, B->x64, n, 1, c->st));
    if (c->verbose) {
      TRY(sync(c));
      std::fprintf(stderr, "wmg setup: level %d vector %d/%d done\n", l, k + 1, nv);
    }
  }
  // the level's operator itself is one full Galerkin build (the same blocks
  // as every other rebuild: load, refresh, given vectors)
  TRY(build_level(c, l, nv));
  c->nl_cur = c->nl;
  return sync(c);
}

static void free_ctx(wmg_ctx *c) {
  if (!c) return;
  for (auto *b : c->batch) free_ctx(b);
  for (int l = 0; l < 3; l++) {
    Level &L = c->lv[l];
    for (int i = 0; i < 3; i++) {
      if (L.U[i]) (void)hipFree(L.U[i]);
      if (L.Uk[i]) (void)hipFree(L.Uk[i]);
      if (L.Ue[i]) (void)hipFree(L.Ue[i]);
    }
    void *ps[] = {L.Y64, L.Y32, L.Ym, L.Ymh, L.Ymsc, L.vecs, L.P64, L.P32, L.P16, L.Ps};
    for (void *p : ps)
      if (p) (void)hipFree(p);
    for (int a = 0; a < 3; a++)
      for (int k = 0; k < NVW; k++)
        if (L.w[a][k]) (void)hipFree(L.w[a][k]);
  }
  for (auto &Bl : c->gb)
  for (auto &B : Bl) {
    for (int k = 0; k < KMAX; k++) {
      if (B.z[k]) (void)hipFree(B.z[k]);
      if (B.wv[k]) (void)hipFree(B.wv[k]);
    }
    void *ps[] = {B.x64, B.r64, B.b64, B.t64, B.zdev, B.wdev};
    for (void *p : ps)
      if (p) (void)hipFree(p);
    if (B.prec != P64 && B.rin) (void)hipFree(B.rin);
  }
  for (auto &kv : c->cg_graphs) {
    if (kv.second.blk) (void)hipGraphExecDestroy(kv.second.blk);
    if (kv.second.tail) (void)hipGraphExecDestroy(kv.second.tail);
  }
  for (auto &e : c->ev_pool) (void)hipEventDestroy(e);
  red_free(c->red);
  if (c->dsc) (void)hipFree(c->dsc);
  if (c->dred) (void)hipFree(c->dred);
  if (c->cpart) (void)hipFree(c->cpart);
  if (c->bpart) (void)hipFree(c->bpart);
  if (c->flag) (void)hipFree(c->flag);
  if (c->hbuf) (void)hipHostFree(c->hbuf);
  if (c->st) (void)hipStreamDestroy(c->st);
  delete c;
}

static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ============================================================ C ABI
extern "C" {

int wmg_default_params(wmg_params *p) {
  if (!p) return set_error(WMG_EINVAL, "null params");
  memset(p, 0, sizeof(*p));
  p->levels = 2;
  for (int l = 0; l < 2; l++)
    for (int i = 0; i < 4; i++) p->block[l][i] = l == 0 ? 4 : 2;
  p->nvec[0] = 24;
  p->nvec[1] = 32;
  p->setup_iters = 5;
  p->post_smooth = 4;
  p->gcr_restart = 8;
  p->cycle = WMG_WCYCLE;
  p->precision = WMG_FP64;
  p->nrhs_max = 1;
  p->coarse_tol = 1e-8;
  p->coarse_maxiter = 500;
  p->reliable_delta = 1e-3;
  p->maxiter = 1000;
  p->seed = 12345;
  p->flags = 0;
  return 0;
}

const char *wmg_strerror(int code) {
  if (g_err[0]) return g_err;
  switch (code) {
    case WMG_OK: return "ok";
    case WMG_ENOTCONV: return "not converged";
    case WMG_EINVAL: return "invalid argument";
    case WMG_ENOMEM: return "out of device memory";
    case WMG_EHIP: return "HIP runtime error";
    case WMG_ERANK: return "block Gram-Schmidt rank breakdown";
    case WMG_EBREAKDOWN: return "numerical breakdown";
  }
  return "unknown error";
}

static int check_geom(const wmg_geom *g) {
  if (!g) return set_error(WMG_EINVAL, "null geometry");
  for (int i = 0; i < 4; i++)
    if (g->L[i] <= 0) return set_error(WMG_EINVAL, "lattice extent L[%d] = %d", i, g->L[i]);
  return 0;
}

static Geom to_geom(const int L[4]) {
  Geom g;
  for (int i = 0; i < 4; i++) g.L[i] = L[i];
  g.V = (long)L[0] * L[1] * L[2] * L[3];
  g.Vs = g.V;
  return g;
}

int wilson_apply(const wmg_geom *g, const double *U, double m, const double *in, double *out, void *hip_stream) {
  g_err[0] = 0;
  TRY(check_geom(g));
  if (!U || !in || !out) return set_error(WMG_EINVAL, "null field pointer");
  if (in == out) return set_error(WMG_EINVAL, "in and out alias");
  return wilson_canonical(to_geom(g->L), U, m, in, out, (hipStream_t)hip_stream);
}

int mg_destroy(wmg_ctx *ctx) {
  free_ctx(ctx);
  return 0;
}

static int ctx_create(const wmg_geom *g, const double *U, double m, int Nv, const int block[4], const wmg_params *pin,
                      wmg_ctx **out) {
  TRY(check_geom(g));
  if (!U || !out || !block) return set_error(WMG_EINVAL, "null argument");
  wmg_params p;
  if (pin) p = *pin;
  else wmg_default_params(&p);
  for (int i = 0; i < 4; i++) p.block[0][i] = block[i];
  p.nvec[0] = Nv;
  if (p.levels < 2 || p.levels > 3) return set_error(WMG_EINVAL, "levels = %d (2 or 3)", p.levels);
  if (p.gcr_restart < 1 || p.gcr_restart > KMAX) return set_error(WMG_EINVAL, "gcr_restart = %d", p.gcr_restart);
  if (p.nrhs_max < 1 || p.nrhs_max > 64) return set_error(WMG_EINVAL, "nrhs_max = %d", p.nrhs_max);
  if (p.flags & WMG_EO_SMOOTHER)
    for (int i = 0; i < 4; i++)
      if (g->L[i] % 2) return set_error(WMG_EINVAL, "red/black smoother needs even extents (L[%d] = %d)", i, g->L[i]);
  int L[4] = {g->L[0], g->L[1], g->L[2], g->L[3]};
  int dof = 12;
  for (int l = 0; l + 1 < p.levels; l++) {
    int bs = 1;
    for (int i = 0; i < 4; i++) {
      if (p.block[l][i] <= 0 || L[i] % p.block[l][i]) 
        return set_error(WMG_EINVAL, "level %d: extent %d not divisible by block %d", l, L[i], p.block[l][i]);
      bs *= p.block[l][i];
    }
    const int ns = (l == 0 && (p.flags & WMG_SPIN_SPLIT)) ? 4 : 2;
    if (p.nvec[l] < 1 || p.nvec[l] > (dof / ns) * bs || p.nvec[l] > 64)
      return set_error(WMG_EINVAL, "level %d: Nv = %d outside [1, %d]", l, p.nvec[l], (dof / ns) * bs < 64 ? (dof / ns) * bs : 64);
    if (ns * p.nvec[l] > 128) return set_error(WMG_EINVAL, "level %d: %d coarse dof > 128", l, ns * p.nvec[l]);
    if (l == 0 && bs > 256) return set_error(WMG_EINVAL, "fine aggregate of %d sites > 256", bs);
    for (int i = 0; i < 4; i++) L[i] /= p.block[l][i];
    dof = ns * p.nvec[l];
  }
  wmg_ctx *c = new wmg_ctx();
  c->p = p;
  c->nl = c->nl_cur = p.levels;
  int rc = 0;
#define CK(x)                  \
  do {                         \
    rc = (x);                  \
    if (rc) goto fail;         \
  } while (0)
  // non-blocking: the default stream (synchronous allocations and fills of
  // other contexts, e.g. the instances of a batch on other host threads)
  // neither waits for this stream nor breaks a graph capture on it
  CK(hipStreamCreateWithFlags(&c->st, hipStreamNonBlocking) == hipSuccess ? 0
                                                                           : set_error(WMG_EHIP, "hipStreamCreate"));
  CK(red_init(c->red, p.nrhs_max));
  CK(dalloc((void **)&c->dsc, sizeof(double) * ((size_t)(4 + 8 + GS + 1) * 64 + 4096)));
  {
    const char *v = std::getenv("WMG_VERBOSE");
    c->verbose = v && *v && *v != '0';
  }
  c->red_out = c->dsc;
  c->cg = c->dsc + 4 * 64;
  c->gcr = c->cg + 8 * 64;
  c->mask = c->gcr + GS * 64;
  c->mr_red = c->mask + 64;          // [4 steps][64 rhs][4]
  c->cyc_nrm = c->mr_red + 4 * 64 * 4;  // [64 rhs][4]
  CK(dalloc((void **)&c->flag, sizeof(int)));
  CK(hipHostMalloc((void **)&c->hbuf, sizeof(double) * 4096) == hipSuccess ? 0 : set_error(WMG_ENOMEM, "hipHostMalloc"));
  {
    Level &F = c->lv[0];
    F.g = to_geom(g->L);
    F.g.Vs = fine_stride(F.g.V);
    F.fine = true;
    F.dof = 12;
    F.n = F.n_alloc = F.g.Vs * 12;
    F.m = m;
    CK(dalloc((void **)&c->dred, sizeof(double) * 3 * (size_t)p.nrhs_max * wilson_red_blocks(F.g)));
    CK(dalloc(&F.U[P64], 16 * 36 * (size_t)F.g.Vs));  // whole links: the Galerkin build reads these
    CK(links_to_soa(F.g, U, P64, F.U[P64], c->st));
    CK(fine_link_format(c, F, U, (p.flags & WMG_LINKS18) != 0));
    for (int l = 0; l + 1 < c->nl; l++) {
      Level &A = c->lv[l], &C = c->lv[l + 1];
      for (int i = 0; i < 4; i++) A.b[i] = p.block[l][i];
      A.nv_max = A.nv = p.nvec[l];
      A.ns = (l == 0 && (p.flags & WMG_SPIN_SPLIT)) ? 4 : 2;
      CK(dalloc((void **)&A.vecs, 16 * (size_t)A.nv_max * A.n));
      CK(dalloc((void **)&A.P64, 16 * (size_t)A.nv_max * A.n));
      int Lc[4];
      for (int i = 0; i < 4; i++) Lc[i] = A.g.L[i] / A.b[i];
      C.g = to_geom(Lc);
      C.fine = false;
      C.dof = C.dof_max = A.ns * A.nv_max;
      C.n = C.n_alloc = C.g.V * C.dof;
      C.m = m;
      CK(dalloc((void **)&C.Y64, 16 * (size_t)C.g.V * 9 * C.dof * C.dof));
    }
  }
  *out = c;
  return 0;
fail:
  free_ctx(c);
  return rc;
#undef CK
}

int mg_setup(const wmg_geom *g, const double *U, double m, int Nv, const int block[4], const wmg_params *p,
             wmg_ctx **out) {
  g_err[0] = 0;
  double t0 = now_s();
  wmg_ctx *c = nullptr;
  TRY(ctx_create(g, U, m, Nv, block, p, &c));
  int rc = 0;
  for (int l = 0; l + 1 < c->nl && !rc; l++) rc = setup_level(c, l);
  if (!rc) rc = make_low_precision(c);
  if (rc) {
    free_ctx(c);
    return rc;
  }
  c->setup_s = now_s() - t0;
  *out = c;
  return 0;
}

int mg_set_mass(wmg_ctx *c, double m) {
  if (!c) return set_error(WMG_EINVAL, "null context");
  if (!c->batch.empty()) return set_error(WMG_EINVAL, "mg_set_mass on a batch context");
  double dm = m - c->lv[0].m;
  for (int l = 0; l < c->nl; l++) c->lv[l].m = m;
  for (int l = 1; l < c->nl; l++) TRY(coarse_shift_diag(c->lv[l].g.V, c->lv[l].dof, c->lv[l].Y64, dm, c->st));
  TRY(sync(c));
  return make_low_precision(c);
}

int mg_solve(wmg_ctx *c, const double *b, double *x, double tol, int nrhs, wmg_stats *stt) {
  g_err[0] = 0;
  if (!c || !b || !x) return set_error(WMG_EINVAL, "null argument");
  if (!c->batch.empty()) return set_error(WMG_EINVAL, "mg_solve on a batch context (use mg_solve_batch)");
  if (nrhs < 1 || nrhs > c->p.nrhs_max) return set_error(WMG_EINVAL, "nrhs = %d outside [1, %d]", nrhs, c->p.nrhs_max);
  if (!(tol > 0)) return set_error(WMG_EINVAL, "tol must be positive");
  double t0 = now_s();
  c->st_fine = c->st_fine64 = c->st_coarse = c->st_rel = 0;
  int ip = c->p.precision == WMG_MIXED ? P32 : P64;
  GcrBuf *B;
  TRY(gcr_buffers(c, 0, ip, nrhs, &B));
  Level &F = c->lv[0];
  TRY(spinor_to_soa(F.g, b, B->b64, nrhs, c->st));
  bool x0 = (c->p.flags & WMG_X0_GIVEN) != 0;
  if (x0) TRY(spinor_to_soa(F.g, x, B->x64, nrhs, c->st));  // else gcr_solve writes x
  double relres = 0;
  double delta = c->p.precision == WMG_MIXED ? c->p.reliable_delta : 0.0;
  int rc = gcr_solve(c, 0, *B, nrhs, tol, c->p.maxiter, 1, delta, x0, c->last_iters, &relres);
  if (rc < 0) return rc;
  TRY(spinor_from_soa(F.g, B->x64, x, nrhs, c->st));
  TRY(sync(c));
  if (stt) {
    int mx = 0;
    for (int v : c->last_iters) mx = v > mx ? v : mx;
    stt->outer_iters = mx;
    stt->fine_matvecs = (int)c->st_fine;
    stt->fine_matvecs_fp64 = (int)c->st_fine64;
    stt->coarse_iters = (int)c->st_coarse;
    stt->reliable_updates = (int)c->st_rel;
    stt->converged = rc == 0;
    stt->true_relres = relres;
    stt->setup_s = c->setup_s;
    stt->solve_s = now_s() - t0;
  }
  return rc;
}

int mg_last_iters(wmg_ctx *c, int *iters, int nrhs) {
  if (!c || !iters) return set_error(WMG_EINVAL, "null argument");
  for (int r = 0; r < nrhs; r++) iters[r] = r < (int)c->last_iters.size() ? c->last_iters[r] : 0;
  return 0;
}

int mg_level_info(wmg_ctx *c, int level, int L[4], int *dof, int *nv) {
  if (!c || level < 0 || level >= c->nl) return set_error(WMG_EINVAL, "level %d", level);
  for (int i = 0; i < 4; i++) L[i] = c->lv[level].g.L[i];
  *dof = c->lv[level].dof;
  *nv = level + 1 < c->nl ? c->lv[level].nv : 0;
  return 0;
}

static int check_level(wmg_ctx *c, int level, bool need_coarse) {
  if (!c) return set_error(WMG_EINVAL, "null context");
  if (level < 0 || level >= c->nl) return set_error(WMG_EINVAL, "level %d", level);
  if (need_coarse && level + 1 >= c->nl) return set_error(WMG_EINVAL, "level %d has no coarser level", level);
  return 0;
}

// canonical [nrhs][V][dof] <-> level vector layout (FP64)
static int to_internal(wmg_ctx *c, int l, const double *canon, double2 *dst, int nrhs) {
  Level &L = c->lv[l];
  if (L.fine) return spinor_to_soa(L.g, canon, dst, nrhs, c->st);
  WMG_HIP(hipMemcpyAsync(dst, canon, 16 * (size_t)L.n * nrhs, hipMemcpyDeviceToDevice, c->st));
  return 0;
}
static int from_internal(wmg_ctx *c, int l, const double2 *src, double *canon, int nrhs) {
  Level &L = c->lv[l];
  if (L.fine) return spinor_from_soa(L.g, src, canon, nrhs, c->st);
  WMG_HIP(hipMemcpyAsync(canon, src, 16 * (size_t)L.n * nrhs, hipMemcpyDeviceToDevice, c->st));
  return 0;
}

int mg_set_null_vectors(wmg_ctx *c, int level, const double *vecs) {
  g_err[0] = 0;
  TRY(check_level(c, level, true));
  if (!vecs) return set_error(WMG_EINVAL, "null vectors");
  Level &F = c->lv[level];
  TRY(to_internal(c, level, vecs, F.vecs, F.nv_max));
  TRY(build_level(c, level, F.nv_max));
  TRY(sync(c));
  return make_low_precision(c);
}

int mg_get_null_vectors(wmg_ctx *c, int level, double *vecs) {
  TRY(check_level(c, level, true));
  Level &F = c->lv[level];
  TRY(from_internal(c, level, F.vecs, vecs, F.nv));
  return sync(c);
}

int mg_get_prolongator(wmg_ctx *c, int level, double *P) {
  TRY(check_level(c, level, true));
  Level &F = c->lv[level];
  void *tmp;
  TRY(dalloc(&tmp, 16 * (size_t)F.nv * F.n));
  int rc = P_block_to_vector(F.g, F.dof, F.b, F.nv, F.P64, (double2 *)tmp, F.fine ? 1 : 0, c->st);
  if (!rc) rc = from_internal(c, level, (double2 *)tmp, P, F.nv);
  if (!rc) rc = sync(c);
  (void)hipFree(tmp);
  return rc;
}

int mg_get_coarse_links(wmg_ctx *c, int level, double *links) {
  TRY(check_level(c, level, false));
  if (level == 0) return set_error(WMG_EINVAL, "level 0 has no coarse links");
  Level &C = c->lv[level];
  TRY(coarse_transpose(C.g.V * 9, C.dof, C.Y64, (double2 *)links, c->st));
  return sync(c);
}

int mg_restrict(wmg_ctx *c, int level, const double *fine, double *coarse, int nrhs) {
  TRY(check_level(c, level, true));
  if (!fine || !coarse || nrhs < 1 || nrhs > c->p.nrhs_max) return set_error(WMG_EINVAL, "bad argument");
  void *tmp;
  TRY(level_vec(c, level, P64, VX, &tmp, nrhs));
  TRY(to_internal(c, level, fine, (double2 *)tmp, nrhs));
  TRY(transfer_restrict(c, level, P64, tmp, coarse, nrhs));
  return sync(c);
}

int mg_prolong(wmg_ctx *c, int level, const double *coarse, double *fine, int nrhs) {
  TRY(check_level(c, level, true));
  if (!fine || !coarse || nrhs < 1 || nrhs > c->p.nrhs_max) return set_error(WMG_EINVAL, "bad argument");
  void *tmp;
  TRY(level_vec(c, level, P64, VX, &tmp, nrhs));
  TRY(transfer_prolong(c, level, P64, coarse, tmp, nrhs));
  TRY(from_internal(c, level, (double2 *)tmp, fine, nrhs));
  return sync(c);
}

int mg_coarse_apply(wmg_ctx *c, int level, const double *in, double *out, int dagger, int nrhs) {
  TRY(check_level(c, level, false));
  if (level == 0) return set_error(WMG_EINVAL, "level 0 is the fine operator");
  if (!in || !out || nrhs < 1 || nrhs > c->p.nrhs_max) return set_error(WMG_EINVAL, "bad argument");
  TRY(apply_op(c, level, P64, in, out, nrhs, false, dagger));
  return sync(c);
}

// ------------------------------------------------------------ setup reuse
// File of a setup: header, then the null vectors of every level in the
// canonical layout [nv][V][dof] (complex128), then an FNV-1a checksum of
// everything before it.  Loading rebuilds P and the coarse operators from
// the vectors for the links given (Sec. 4: the setup is amortised over
// many solves and, as U evolves, refreshed instead of redone).
struct SetupFileHeader {
  char magic[8];      // "WMGSETUP"
  int version;        // 1
  int L[4];
  int levels;
  int nv[2];
  int dof[2];         // per-site dof of levels 0 and 1
  long V[2];          // sites of levels 0 and 1
  double mass;
  wmg_params params;
};

static uint64_t fnv1a(uint64_t h, const void *p, size_t n) {
  const unsigned char *b = (const unsigned char *)p;
  for (size_t i = 0; i < n; i++) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}

static int read_setup_file(const char *path, SetupFileHeader &h, std::vector<std::vector<double>> &vecs) {
  FILE *f = std::fopen(path, "rb");
  if (!f) return set_error(WMG_EINVAL, "mg_load: cannot open %s", path);
  int rc = 0;
  uint64_t sum = 1469598103934665603ull, stored = 0;
  if (std::fread(&h, sizeof(h), 1, f) != 1 || std::memcmp(h.magic, "WMGSETUP", 8) || h.version != 1 ||
      h.levels < 2 || h.levels > 3)
    rc = set_error(WMG_EINVAL, "mg_load: %s is not a setup file of this library", path);
  sum = fnv1a(sum, &h, sizeof(h));
  for (int l = 0; !rc && l + 1 < h.levels; l++) {
    if (h.nv[l] < 1 || h.nv[l] > 64 || h.dof[l] < 1 || h.V[l] < 1 || h.V[l] > (1L << 34)) {
      rc = set_error(WMG_EINVAL, "mg_load: %s: bad level %d sizes", path, l);
      break;
    }
    vecs.emplace_back((size_t)h.nv[l] * h.V[l] * h.dof[l] * 2);
    auto &v = vecs.back();
    if (std::fread(v.data(), sizeof(double), v.size(), f) != v.size()) {
      rc = set_error(WMG_EINVAL, "mg_load: %s is truncated", path);
      break;
    }
    sum = fnv1a(sum, v.data(), sizeof(double) * v.size());
  }
  if (!rc && std::fread(&stored, sizeof(stored), 1, f) != 1) rc = set_error(WMG_EINVAL, "mg_load: %s is truncated", path);
  if (!rc && stored != sum) rc = set_error(WMG_EINVAL, "mg_load: %s fails its checksum", path);
  std::fclose(f);
  return rc;
}

// rebuild every level from the null vectors in F.vecs (levels in order:
// level l's vectors live on the operator that level l-1 built)
static int rebuild_all(wmg_ctx *c) {
  for (int l = 0; l + 1 < c->nl; l++) TRY(build_level(c, l, c->lv[l].nv_max));
  TRY(sync(c));
  return make_low_precision(c);
}

// Improve every null vector of level l by `iters` steps of GCR on A x = 0,
// preconditioned with the current hierarchy, starting from the vector
// itself; then normalise.  Levels above l must already be built for the
// current links.
static int refresh_level(wmg_ctx *c, int l, int iters) {
  Level &F = c->lv[l];
  GcrBuf *B;
  TRY(gcr_buffers(c, l, P64, 1, &B));
  std::vector<int> its;
  const long n = F.n;
  for (int k = 0; k < F.nv_max; k++) {
    TRY(copy(P64, B->x64, P64, F.vecs + (size_t)k * n, n, 1, c->st));
    TRY(zero(P64, B->b64, n, 1, c->st));
    int rc = gcr_solve(c, l, *B, 1, 0.0, iters, 1, 0.0, true, its, nullptr);
    if (rc < 0) return rc;
    TRY(norm2(c->red, P64, B->x64, n, 1, c->red_out, 4, c->st));
    TRY(scale_inv_sqrt(P64, B->x64, c->red_out, 4, n, 1, c->st));
    TRY(copy(P64, F.vecs + (size_t)k * n, P64, B->x64, n, 1, c->st));
  }
  return sync(c);
}

int mg_save(wmg_ctx *c, const char *path) {
  g_err[0] = 0;
  if (!c || !path) return set_error(WMG_EINVAL, "null argument");
  if (!c->batch.empty()) return set_error(WMG_EINVAL, "mg_save on a batch context");
  SetupFileHeader h;
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, "WMGSETUP", 8);
  h.version = 1;
  for (int i = 0; i < 4; i++) h.L[i] = c->lv[0].g.L[i];
  h.levels = c->nl;
  for (int l = 0; l + 1 < c->nl; l++) {
    h.nv[l] = c->lv[l].nv_max;
    h.dof[l] = c->lv[l].dof;
    h.V[l] = c->lv[l].g.V;
  }
  h.mass = c->lv[0].m;
  h.params = c->p;
  FILE *f = std::fopen(path, "wb");
  if (!f) return set_error(WMG_EINVAL, "mg_save: cannot create %s", path);
  uint64_t sum = fnv1a(1469598103934665603ull, &h, sizeof(h));
  int rc = std::fwrite(&h, sizeof(h), 1, f) == 1 ? 0 : set_error(WMG_EINVAL, "mg_save: write to %s failed", path);
  for (int l = 0; !rc && l + 1 < c->nl; l++) {
    Level &F = c->lv[l];
    const size_t cnt = (size_t)F.nv_max * F.g.V * F.dof;
    double *tmp = nullptr;
    rc = dalloc((void **)&tmp, 16 * cnt);
    if (!rc) rc = from_internal(c, l, F.vecs, tmp, F.nv_max);
    std::vector<double> hv(2 * cnt);
    if (!rc && hipMemcpyAsync(hv.data(), tmp, 16 * cnt, hipMemcpyDeviceToHost, c->st) != hipSuccess)
      rc = set_error(WMG_EHIP, "mg_save: read-back");
    if (!rc) rc = sync(c);
    if (tmp) (void)hipFree(tmp);
    if (!rc && std::fwrite(hv.data(), sizeof(double), hv.size(), f) != hv.size())
      rc = set_error(WMG_EINVAL, "mg_save: write to %s failed", path);
    sum = fnv1a(sum, hv.data(), sizeof(double) * hv.size());
  }
  if (!rc && std::fwrite(&sum, sizeof(sum), 1, f) != 1) rc = set_error(WMG_EINVAL, "mg_save: write to %s failed", path);
  if (std::fclose(f) && !rc) rc = set_error(WMG_EINVAL, "mg_save: closing %s failed", path);
  return rc;
}

int mg_load(const char *path, const wmg_geom *g, const double *U, double m, const wmg_params *p, wmg_ctx **out) {
  g_err[0] = 0;
  if (!path || !g || !U || !out) return set_error(WMG_EINVAL, "null argument");
  SetupFileHeader h;
  std::vector<std::vector<double>> vecs;
  TRY(read_setup_file(path, h, vecs));
  for (int i = 0; i < 4; i++)
    if (g->L[i] != h.L[i])
      return set_error(WMG_EINVAL, "mg_load: lattice %dx%dx%dx%d, the file holds %dx%dx%dx%d", g->L[0], g->L[1],
                       g->L[2], g->L[3], h.L[0], h.L[1], h.L[2], h.L[3]);
  wmg_params q = h.params;
  if (p) {
    // solver settings may change; the hierarchy's shape must not
    bool same = p->levels == h.params.levels;
    for (int l = 0; same && l + 1 < h.levels; l++) {
      same = same && p->nvec[l] == h.params.nvec[l];
      for (int i = 0; i < 4 && l > 0; i++) same = same && p->block[l][i] == h.params.block[l][i];
    }
    if (!same) return set_error(WMG_EINVAL, "mg_load: parameters describe another hierarchy than %s", path);
    q = *p;
    q.block[0][0] = h.params.block[0][0];  // block[0] and nvec[0] come from the file
    for (int i = 0; i < 4; i++) q.block[0][i] = h.params.block[0][i];
  }
  double t0 = now_s();
  wmg_ctx *c = nullptr;
  TRY(ctx_create(g, U, m, h.nv[0], h.params.block[0], &q, &c));
  int rc = 0;
  for (int l = 0; !rc && l + 1 < c->nl; l++) {
    Level &F = c->lv[l];
    if (F.nv_max != h.nv[l] || F.dof != h.dof[l] || F.g.V != h.V[l]) {
      rc = set_error(WMG_EINVAL, "mg_load: level %d of %s does not match the parameters", l, path);
      break;
    }
    double *tmp = nullptr;
    const size_t cnt = (size_t)F.nv_max * F.g.V * F.dof;
    rc = dalloc((void **)&tmp, 16 * cnt);
    if (!rc && hipMemcpyAsync(tmp, vecs[l].data(), 16 * cnt, hipMemcpyHostToDevice, c->st) != hipSuccess)
      rc = set_error(WMG_EHIP, "mg_load: upload");
    if (!rc) rc = to_internal(c, l, tmp, F.vecs, F.nv_max);
    if (!rc) rc = sync(c);
    if (tmp) (void)hipFree(tmp);
    if (!rc) rc = build_level(c, l, F.nv_max);  // the next level's vectors live on this operator
  }
  if (!rc) rc = sync(c);
  if (!rc) rc = make_low_precision(c);
  if (rc) {
    free_ctx(c);
    return rc;
  }
  c->setup_s = now_s() - t0;
  *out = c;
  return 0;
}

int mg_refresh(wmg_ctx *c, const double *U, int iters) {
  g_err[0] = 0;
  if (!c || !U || iters < 0) return set_error(WMG_EINVAL, "bad argument");
  if (!c->batch.empty()) return set_error(WMG_EINVAL, "mg_refresh on a batch context");
  double t0 = now_s();
  Level &F = c->lv[0];
  // new links in every format the context keeps
  TRY(links_to_soa(F.g, U, P64, F.U[P64], c->st));
  for (int lp = P64; lp <= P16; lp++) {
    if (F.Ue[lp]) (void)hipFree(F.Ue[lp]);
    F.Ue[lp] = nullptr;
    if (F.Uk[lp]) (void)hipFree(F.Uk[lp]);
    if (lp != P64 && F.U[lp]) (void)hipFree(F.U[lp]);
    F.Uk[lp] = nullptr;
    if (lp != P64) F.U[lp] = nullptr;
  }
  TRY(fine_link_format(c, F, U, (c->p.flags & WMG_LINKS18) != 0));
  // Galerkin operators for the new links from the old vectors, then each
  // level's vectors relaxed with that hierarchy and the level rebuilt
  TRY(rebuild_all(c));
  if (iters > 0)
    for (int l = 0; l + 1 < c->nl; l++) {
      TRY(refresh_level(c, l, iters));
      for (int k = l; k + 1 < c->nl; k++) TRY(build_level(c, k, c->lv[k].nv_max));
      TRY(sync(c));
      TRY(make_low_precision(c));
    }
  c->setup_s = now_s() - t0;
  return 0;
}

// restriction (dir 0) or prolongation (dir 1) through the FP32 vectors and
// FP16-stored prolongator of a mixed-precision context
static int transfer_f32(wmg_ctx *c, int level, int dir, const double *in, double *out, int nrhs) {
  TRY(check_level(c, level, true));
  if (!in || !out || nrhs < 1 || nrhs > c->p.nrhs_max) return set_error(WMG_EINVAL, "bad argument");
  if (c->p.precision != WMG_MIXED) return set_error(WMG_EINVAL, "FP16 prolongator exists in mixed precision only");
  Level &F = c->lv[level], &C = c->lv[level + 1];
  void *f32, *c32, *f64;
  TRY(level_vec(c, level, P32, VX, &f32, nrhs));
  TRY(level_vec(c, level + 1, P32, VX, &c32, nrhs));
  TRY(level_vec(c, level, P64, VX, &f64, nrhs));
  if (dir == 0) {
    TRY(to_internal(c, level, in, (double2 *)f64, nrhs));
    TRY(copy(P32, f32, P64, f64, F.n, nrhs, c->st));
    // as the mixed cycle runs it: on the fine level with |in|^2 per rhs
    double *nrm = nullptr;
    if (F.fine) {
      TRY(cpart_get(c, 4 * (size_t)nrhs, &nrm));
      TRY(norm2(c->red, P32, f32, F.n, nrhs, nrm, 4, c->st));
    }
    TRY(transfer_restrict(c, level, P32, f32, c32, nrhs, nrm));
    TRY(copy(P64, out, P32, c32, C.n, nrhs, c->st));
  } else {
    TRY(copy(P32, c32, P64, in, C.n, nrhs, c->st));
    TRY(transfer_prolong(c, level, P32, c32, f32, nrhs));
    TRY(copy(P64, f64, P32, f32, F.n, nrhs, c->st));
    TRY(from_internal(c, level, (double2 *)f64, out, nrhs));
  }
  return sync(c);
}

int mg_restrict_f32(wmg_ctx *c, int level, const double *fine, double *coarse, int nrhs) {
  return transfer_f32(c, level, 0, fine, coarse, nrhs);
}
int mg_prolong_f32(wmg_ctx *c, int level, const double *coarse, double *fine, int nrhs) {
  return transfer_f32(c, level, 1, coarse, fine, nrhs);
}

int mg_coarse_apply_f32(wmg_ctx *c, int level, const double *in, double *out, int dagger, int nrhs) {
  TRY(check_level(c, level, false));
  if (level == 0) return set_error(WMG_EINVAL, "level 0 is the fine operator");
  if (!in || !out || nrhs < 1 || nrhs > c->p.nrhs_max) return set_error(WMG_EINVAL, "bad argument");
  if (c->p.precision != WMG_MIXED) return set_error(WMG_EINVAL, "FP32 coarse operator exists in mixed precision only");
  Level &C = c->lv[level];
  void *a, *b;
  TRY(level_vec(c, level, P32, VX, &a, nrhs));
  TRY(level_vec(c, level, P32, VT, &b, nrhs));
  TRY(copy(P32, a, P64, in, C.n, nrhs, c->st));
  TRY(apply_op(c, level, P32, a, b, nrhs, false, dagger));
  TRY(copy(P64, out, P32, b, C.n, nrhs, c->st));
  return sync(c);
}

int mg_apply_fine(wmg_ctx *c, int prec, const double *in, double *out, int nrhs) {
  if (!c || !in || !out || nrhs < 1 || nrhs > c->p.nrhs_max || nrhs > 64 || prec < 0 || prec > 4)
    return set_error(WMG_EINVAL, "bad argument");
  Level &F = c->lv[0];
  void *a64, *b64;
  TRY(level_vec(c, 0, P64, VX, &a64, nrhs));
  TRY(level_vec(c, 0, P64, VT, &b64, nrhs));
  TRY(spinor_to_soa(F.g, in, (double2 *)a64, nrhs, c->st));
  if (prec == 0) {
    TRY(wilson_soa(F.g, fine_lcode(F, P64), fine_links(F, P64), P64, F.m, a64, b64, nrhs, c->st));
  } else if (prec == 4) {
    // the inner GCR's operator on an FP16-stored field: in rounded to FP16,
    // FP32 links and arithmetic, FP32 output
    if (F.n % 4) return set_error(WMG_EINVAL, "length not a multiple of 4");
    void *a32, *h, *b32;
    TRY(level_vec(c, 0, P32, VX, &a32, nrhs));
    TRY(level_vec(c, 0, P32, VT, &b32, nrhs));
    TRY(level_vec(c, 0, P16, VS, &h, nrhs));
    TRY(copy(P32, a32, P64, a64, F.n, nrhs, c->st));
    TRY(copy(P16, h, P32, a32, F.n, nrhs, c->st));
    TRY(wilson_soa_in16(F.g, fine_lcode(F, P32), fine_links(F, P32), F.m, h, b32, nrhs, c->st));
    TRY(copy(P64, b64, P32, b32, F.n, nrhs, c->st));
  } else if (prec < 3) {
    void *a32, *b32;
    TRY(level_vec(c, 0, P32, VX, &a32, nrhs));
    TRY(level_vec(c, 0, P32, VT, &b32, nrhs));
    TRY(copy(P32, a32, P64, a64, F.n, nrhs, c->st));
    const int lp = prec == 1 ? P32 : P16;
    TRY(wilson_soa(F.g, fine_lcode(F, lp), fine_links(F, lp), P32, F.m, a32, b32, nrhs, c->st));
    TRY(copy(P64, b64, P32, b32, F.n, nrhs, c->st));
  } else {
    // the MR step's operator: in/|in| stored in FP16 by the smoother's
    // residual kernel (with e = 0), then FP16 links on FP16 spinors, FP16
    // output; returned as FP64 times |in|
    if (F.n % 4) return set_error(WMG_EINVAL, "length not a multiple of 4");
    void *a32, *e32, *h0, *h1, *b32;
    TRY(level_vec(c, 0, P32, VX, &a32, nrhs));
    TRY(level_vec(c, 0, P32, VE, &e32, nrhs));
    TRY(level_vec(c, 0, P32, VT, &b32, nrhs));
    TRY(level_vec(c, 0, P16, VS, &h0, nrhs));
    TRY(level_vec(c, 0, P16, VQ, &h1, nrhs));
    TRY(copy(P32, a32, P64, a64, F.n, nrhs, c->st));
    TRY(zero(P32, e32, F.n, nrhs, c->st));
    double *rn2 = c->cyc_nrm;
    TRY(norm2(c->red, P32, a32, F.n, nrhs, rn2, 4, c->st));
    TRY(wilson_soa_h16(F.g, fine_links(F, P16), P32, F.m, e32, h0, nrhs, a32, rn2, 4, nullptr, nullptr, 0, c->st,
                       F.lk));
    TRY(wilson_soa_h16(F.g, fine_links(F, P16), P16, F.m, h0, h1, nrhs, nullptr, nullptr, 0, nullptr, nullptr, 0,
                       c->st, F.lk));
    TRY(copy(P32, b32, P16, h1, F.n, nrhs, c->st));
    TRY(scale_sqrt(P32, b32, rn2, 4, F.n, nrhs, c->st));
    TRY(copy(P64, b64, P32, b32, F.n, nrhs, c->st));
  }
  TRY(spinor_from_soa(F.g, (double2 *)b64, out, nrhs, c->st));
  return sync(c);
}

// canonical FP64 full-lattice vectors -> half-lattice arrays (even, odd) of
// precision p, through the fine level's work vectors VX / VS
static int canon_to_eo(wmg_ctx *c, int p, const double *canon, void *ev, void *od, int nrhs) {
  Level &F = c->lv[0];
  void *a64;
  TRY(level_vec(c, 0, P64, VX, &a64, nrhs));
  TRY(spinor_to_soa(F.g, canon, (double2 *)a64, nrhs, c->st));
  if (p == P64) return eo_pack(F.g, P64, a64, P64, ev, od, nrhs, c->st);
  void *a32;
  TRY(level_vec(c, 0, P32, VX, &a32, nrhs));
  TRY(copy(P32, a32, P64, a64, F.n, nrhs, c->st));
  if (p == P32) return eo_pack(F.g, P32, a32, P32, ev, od, nrhs, c->st);
  void *a16;
  TRY(level_vec(c, 0, P16, VS, &a16, nrhs));
  TRY(copy(P16, a16, P32, a32, F.n, nrhs, c->st));
  return eo_pack(F.g, P16, a16, P16, ev, od, nrhs, c->st);
}

int mg_hop_eo(wmg_ctx *c, int prec, int par, double a, double b, const double *diag, const double *hop, double *out,
              int nrhs) {
  if (!c || !hop || !out || (a != 0.0 && !diag) || nrhs < 1 || nrhs > c->p.nrhs_max || nrhs > 64 ||
      (prec != 0 && prec != 3 && prec != 4 && prec != 5 && prec != 6) || (par != 0 && par != 1) ||
      (prec >= 5 && par != 1))
    return set_error(WMG_EINVAL, "bad argument");
  Level &F = c->lv[0];
  for (int i = 0; i < 4; i++)
    if (F.g.L[i] % 2) return set_error(WMG_EINVAL, "red/black sublattices need even extents");
  const int lp = prec == 0 ? P64 : P16;                        // links
  const int pd = prec == 0 ? P64 : P16;                        // diag
  const int ph = prec == 0 ? P64 : (prec == 4 ? P32 : P16);    // hop input (and output, prec 0, 3, 4)
  const void *Ue;
  TRY(eo_links(c, lp, &Ue));
  void *de, *dod, *he, *ho, *o;
  TRY(level_vec(c, 0, pd, VHSE, &de, nrhs));
  TRY(level_vec(c, 0, pd, VHSO, &dod, nrhs));
  TRY(level_vec(c, 0, ph, VHDE, &he, nrhs));
  TRY(level_vec(c, 0, ph, VHDO, &ho, nrhs));
  TRY(level_vec(c, 0, ph, VHQ, &o, nrhs));
  if (a != 0.0) TRY(canon_to_eo(c, pd, diag, de, dod, nrhs));
  TRY(canon_to_eo(c, ph, hop, he, ho, nrhs));
  const long nh = 12 * eo_stride(F.g);
  const int pf = prec == 0 ? P64 : P32;
  void *full, *b64;
  TRY(level_vec(c, 0, pf, VT, &full, nrhs));
  TRY(zero(pf, full, F.n, nrhs, c->st));
  if (prec >= 5) {
    // the smoother's last step as the mixed cycle runs it: full = base +
    // (hop at the even sites, the odd result), here with a zero FP16 base;
    // prec 6 stores full in FP16
    void *base;
    TRY(level_vec(c, 0, P16, VEH, &base, nrhs));
    TRY(zero(P16, base, F.n, nrhs, c->st));
    if (prec == 6) {
      void *f16;
      TRY(level_vec(c, 0, P16, VS, &f16, nrhs));
      TRY(hop_eo_add(F.g, lp | F.lk, Ue, a, b, pd, a != 0.0 ? dod : nullptr, ph, he, f16, nrhs, c->st, base, P16));
      TRY(copy(P32, full, P16, f16, F.n, nrhs, c->st));
    } else {
      TRY(hop_eo_add(F.g, lp | F.lk, Ue, a, b, pd, a != 0.0 ? dod : nullptr, ph, he, full, nrhs, c->st, base));
    }
  } else {
    TRY(hop_eo(F.g, lp | F.lk, Ue, par, a, b, pd, a != 0.0 ? (par ? dod : de) : nullptr, ph, par ? he : ho, ph, o,
               nrhs, nullptr, nullptr, 0, c->st));
    // result (sites of parity par) -> zeroed full lattice
    void *o2 = o;
    if (ph == P16) {
      TRY(level_vec(c, 0, P32, VHQ, &o2, nrhs));
      TRY(copy(P32, o2, P16, o, nh, nrhs, c->st));
    }
    TRY(eo_unpack_add(F.g, pf, full, pf, par ? nullptr : o2, par ? o2 : nullptr, nrhs, c->st));
  }
  b64 = full;
  if (pf == P32) {
    TRY(level_vec(c, 0, P64, VT, &b64, nrhs));
    TRY(copy(P64, b64, P32, full, F.n, nrhs, c->st));
  }
  TRY(spinor_from_soa(F.g, (double2 *)b64, out, nrhs, c->st));
  return sync(c);
}

int mg_smoother_residual(wmg_ctx *c, const double *r, const double *e, double *out, int nrhs) {
  if (!c || !r || !e || !out || nrhs < 1 || nrhs > c->p.nrhs_max || nrhs > 64) return set_error(WMG_EINVAL, "bad argument");
  Level &F = c->lv[0];
  if (F.n % 4) return set_error(WMG_EINVAL, "length not a multiple of 4");
  void *a64, *r32, *e32, *h0, *b32;
  TRY(level_vec(c, 0, P64, VX, &a64, nrhs));
  TRY(level_vec(c, 0, P32, VX, &r32, nrhs));
  TRY(level_vec(c, 0, P32, VE, &e32, nrhs));
  TRY(level_vec(c, 0, P32, VT, &b32, nrhs));
  TRY(level_vec(c, 0, P16, VS, &h0, nrhs));
  TRY(spinor_to_soa(F.g, r, (double2 *)a64, nrhs, c->st));
  TRY(copy(P32, r32, P64, a64, F.n, nrhs, c->st));
  TRY(spinor_to_soa(F.g, e, (double2 *)a64, nrhs, c->st));
  TRY(copy(P32, e32, P64, a64, F.n, nrhs, c->st));
  double *rn2 = c->cyc_nrm;
  TRY(norm2(c->red, P32, r32, F.n, nrhs, rn2, 4, c->st));
  if ((c->p.flags & WMG_EO_SMOOTHER) && prolong16_ok(c, 0, nrhs)) {
    // the red/black smoother's form: e in FP16, the result in the two
    // half-lattice arrays
    void *eh, *se, *so, *se32, *so32;
    TRY(level_vec(c, 0, P16, VEH, &eh, nrhs));
    TRY(level_vec(c, 0, P16, VHSE, &se, nrhs));
    TRY(level_vec(c, 0, P16, VHSO, &so, nrhs));
    TRY(level_vec(c, 0, P32, VHSE, &se32, nrhs));
    TRY(level_vec(c, 0, P32, VHSO, &so32, nrhs));
    const long nh = 12 * eo_stride(F.g);
    TRY(copy(P16, eh, P32, e32, F.n, nrhs, c->st));
    TRY(wilson_soa_h16(F.g, fine_links(F, P16), P16, F.m, eh, se, nrhs, r32, rn2, 4, nullptr, nullptr, 0, c->st,
                       F.lk, so));
    TRY(copy(P32, se32, P16, se, nh, nrhs, c->st));
    TRY(copy(P32, so32, P16, so, nh, nrhs, c->st));
    TRY(zero(P32, b32, F.n, nrhs, c->st));
    TRY(eo_unpack_add(F.g, P32, b32, P32, se32, so32, nrhs, c->st));
  } else {
    TRY(wilson_soa_h16(F.g, fine_links(F, P16), P32, F.m, e32, h0, nrhs, r32, rn2, 4, nullptr, nullptr, 0, c->st,
                       F.lk));
    TRY(copy(P32, b32, P16, h0, F.n, nrhs, c->st));
  }
  TRY(copy(P64, a64, P32, b32, F.n, nrhs, c->st));
  TRY(spinor_from_soa(F.g, (double2 *)a64, out, nrhs, c->st));
  return sync(c);
}

int mg_cycle(wmg_ctx *c, const double *r, double *z) {
  if (!c || !r || !z) return set_error(WMG_EINVAL, "bad argument");
  Level &F = c->lv[0];
  void *a, *e;
  TRY(level_vec(c, 0, P64, VX, &a, 1));
  TRY(level_vec(c, 0, P64, VE2, &e, 1));
  TRY(spinor_to_soa(F.g, r, (double2 *)a, 1, c->st));
  TRY(mg_cycle_l(c, 0, P64, a, e, 1));
  TRY(spinor_from_soa(F.g, (double2 *)e, z, 1, c->st));
  return sync(c);
}

int mg_time_dslash(wmg_ctx *c, int prec, int nrhs, int reps, double *ms) {
  if (!c || !ms || nrhs < 1 || nrhs > c->p.nrhs_max || reps < 1 || prec < 0 || prec > 2)
    return set_error(WMG_EINVAL, "bad argument");
  Level &F = c->lv[0];
  int sp = prec == 0 ? P64 : P32;
  int lp = prec == 0 ? P64 : (prec == 1 ? P32 : P16);
  void *a, *b;
  TRY(level_vec(c, 0, sp, VX, &a, nrhs));
  TRY(level_vec(c, 0, sp, VT, &b, nrhs));
  void *a64;
  TRY(level_vec(c, 0, P64, VE2, &a64, 1));
  TRY(start_vectors(F.g.V, 12, 99, 7, 0, 1, (double2 *)a64, 1, F.g.Vs, c->st));
  for (int r = 0; r < nrhs; r++) TRY(copy(sp, (char *)a + csize(sp) * (size_t)F.n * r, P64, a64, F.n, 1, c->st));
  TRY(wilson_soa(F.g, fine_lcode(F, lp), fine_links(F, lp), sp, F.m, a, b, nrhs, c->st));  // warm-up
  hipEvent_t e0, e1;
  WMG_HIP(hipEventCreate(&e0));
  WMG_HIP(hipEventCreate(&e1));
  WMG_HIP(hipEventRecord(e0, c->st));
  for (int i = 0; i < reps; i++)
    TRY(wilson_soa(F.g, fine_lcode(F, lp), fine_links(F, lp), sp, F.m, (i & 1) ? b : a, (i & 1) ? a : b, nrhs, c->st));
  WMG_HIP(hipEventRecord(e1, c->st));
  WMG_HIP(hipEventSynchronize(e1));
  float t = 0;
  WMG_HIP(hipEventElapsedTime(&t, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = t / reps;
  return 0;
}

int mg_link_reals(wmg_ctx *c) {
  if (!c) return set_error(WMG_EINVAL, "null context");
  if (!c->batch.empty()) return mg_link_reals(c->batch[0]);
  return c->lv[0].lk ? 12 : 18;
}

int mg_set_precision(wmg_ctx *c, int precision) {
  if (!c || (precision != WMG_FP64 && precision != WMG_MIXED)) return set_error(WMG_EINVAL, "bad argument");
  c->p.precision = precision;
  return make_low_precision(c);
}

int mg_profile(wmg_ctx *c, int enable) {
  if (!c) return set_error(WMG_EINVAL, "null context");
  TRY(prof_resolve(c));
  c->prof = enable != 0;
  for (int k = 0; k < 8; k++) {
    c->prof_ms[k] = c->prof_bytes[k] = 0;
    c->prof_n[k] = 0;
  }
  return 0;
}

int mg_profile_get(wmg_ctx *c, int kind, int *launches, double *total_ms, double *total_bytes) {
  if (!c || kind < 0 || kind >= K_NKIND || !launches || !total_ms || !total_bytes)
    return set_error(WMG_EINVAL, "bad argument");
  TRY(prof_resolve(c));
  *launches = (int)c->prof_n[kind];
  *total_ms = c->prof_ms[kind];
  *total_bytes = c->prof_bytes[kind];
  return 0;
}

// ------------------------------------------------------------ batch
// Uneven batch: one context (own stream, own buffers) per instance; setup
// and solve of all instances are driven from one host thread each, so the
// instances' kernels run concurrently on the device and small lattices
// fill the GPU together.
int mg_setup_batch(int n, const wmg_geom *g, const double *const *U, const double *m, int Nv, const int block[4],
                   const wmg_params *p, wmg_ctx **out) {
  g_err[0] = 0;
  if (n < 1 || n > 256 || !g || !U || !m || !out || !block) return set_error(WMG_EINVAL, "bad argument");
  wmg_ctx *parent = new wmg_ctx();
  if (p) parent->p = *p;
  else wmg_default_params(&parent->p);
  // the instances run on concurrent host threads, whose allocations and
  // synchronisations a stream capture on one of them does not tolerate:
  // no graph capture inside a batch
  wmg_params pi = parent->p;
  pi.flags &= ~WMG_GRAPHS;
  std::vector<wmg_ctx *> ctx(n, nullptr);
  std::vector<int> rcs(n, 0);
  std::vector<std::string> msgs(n);
  std::vector<std::thread> th;
  for (int i = 0; i < n; i++)
    th.emplace_back([&, i]() {
      rcs[i] = mg_setup(&g[i], U[i], m[i], Nv, block, &pi, &ctx[i]);
      if (rcs[i]) msgs[i] = g_err;
    });
  for (auto &t : th) t.join();
  int rc = 0;
  for (int i = 0; i < n; i++) {
    if (ctx[i]) parent->batch.push_back(ctx[i]);
    if (rcs[i] && !rc) {
      rc = rcs[i];
      set_error(rc, "instance %d: %s", i, msgs[i].c_str());
    }
  }
  if (rc) {
    free_ctx(parent);
    return rc;
  }
  *out = parent;
  return 0;
}

int mg_solve_batch(wmg_ctx *c, const double *const *b, double *const *x, double tol, wmg_stats *st) {
  g_err[0] = 0;
  if (!c || c->batch.empty() || !b || !x) return set_error(WMG_EINVAL, "not a batch context");
  int n = (int)c->batch.size();
  std::vector<int> rcs(n, 0);
  std::vector<std::string> msgs(n);
  std::vector<std::thread> th;
  for (int i = 0; i < n; i++)
    th.emplace_back([&, i]() {
      rcs[i] = mg_solve(c->batch[i], b[i], x[i], tol, 1, st ? &st[i] : nullptr);
      if (rcs[i]) msgs[i] = g_err;
    });
  for (auto &t : th) t.join();
  int worst = 0;
  for (int i = 0; i < n; i++) {
    if (rcs[i] < 0) return set_error(rcs[i], "instance %d: %s", i, msgs[i].c_str());
    if (rcs[i] > worst) worst = rcs[i];
  }
  return worst;
}

}  // extern "C"
