// Unpreconditioned BiCGStab on the Wilson operator: the unigrid Krylov
// baseline against which the multigrid solve is compared (the paper compares
// MG with unigrid CG-type solvers in Fig. 2-3).  FP64, one right-hand side,
// internal SoA layouts; scalars are read back to the host every iteration.
#include <cmath>
#include <mutex>
#include <vector>

#include "wmg_internal.h"
#include "../../include/wmg.h"

using namespace wmg;

namespace {
struct H {
  double re, im;
};
H hmul(H a, H b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
H hdiv(H a, H b) {
  double d = b.re * b.re + b.im * b.im;
  return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}
}  // namespace

// Work buffers of one BiCGStab solve: SoA links, eight fine vectors, 64
// device scalars and the reduction partials.  Padding sites of every vector
// must be zero on entry.
struct BiWork {
  void *Us;
  double2 *x, *b, *r, *rh, *p, *v, *sv, *t;
  double *dsc;
  Reducer R;
};

// hb: 64 host doubles for scalar read-back and coefficient upload (each
// coefficient has its own slot: the uploads are asynchronous)
static int bicgstab_run(const Geom &g, const double *U, double m, const double *bc, double *xc, double tol,
                        int maxiter, wmg_stats *st, hipStream_t s, BiWork &w, double *hb) {
  long n = g.Vs * 12;
  int rc = 0, it = 0;
  double relres = 0;
  Reducer &R = w.R;
  double2 *x = w.x, *b = w.b, *r = w.r, *rh = w.rh, *p = w.p, *v = w.v, *sv = w.sv, *t = w.t;
  double *dsc = w.dsc;
  void *Us = w.Us;
#define C(x)            \
  do {                  \
    rc = (x);           \
    if (rc) return rc;  \
  } while (0)
#define RD()                                                                                       \
  do {                                                                                             \
    if (hipMemcpyAsync(hb, dsc, sizeof(double) * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||    \
        hipStreamSynchronize(s) != hipSuccess)                                                     \
      return set_error(WMG_EHIP, "readback");                                                      \
  } while (0)
  C(links_to_soa(g, U, P64, Us, s));
  C(spinor_to_soa(g, bc, b, 1, s));
  C(zero(P64, x, n, 1, s));
  C(copy(P64, r, P64, b, n, 1, s));
  C(copy(P64, rh, P64, b, n, 1, s));
  C(zero(P64, p, n, 1, s));
  C(zero(P64, v, n, 1, s));
  C(norm2(R, P64, b, n, 1, dsc, 4, s));
  RD();
  double bn = sqrt(hb[0]), rn = bn;
  H rho = {1, 0}, al = {1, 0}, om = {1, 0};
  double *coef = dsc + 16;  // device coefficient slots (re, im)
  while (rn > tol * bn && it < maxiter) {
    C(dot(R, P64, rh, r, n, 1, dsc, 4, s));
    RD();
    H rho1 = {hb[0], hb[1]};
    if (rho1.re == 0 && rho1.im == 0) break;
    H be = hmul(hdiv(rho1, rho), hdiv(al, om));
    // p = r + be (p - om v)
    hb[16] = -om.re; hb[17] = -om.im; hb[18] = be.re; hb[19] = be.im;
    C(hipMemcpyAsync(coef, hb + 16, 32, hipMemcpyHostToDevice, s) == hipSuccess ? 0 : -3);
    C(caxpy_dev(P64, coef, 0, 1.0, v, p, n, 1, s));
    C(cxpay_dev(P64, r, coef + 2, 0, 1.0, p, n, 1, s));
    C(wilson_soa(g, P64, Us, P64, m, p, v, 1, s));
    C(dot(R, P64, rh, v, n, 1, dsc, 4, s));
    RD();
    al = hdiv(rho1, H{hb[0], hb[1]});
    // s = r - al v
    C(copy(P64, sv, P64, r, n, 1, s));
    hb[20] = -al.re; hb[21] = -al.im;
    C(hipMemcpyAsync(coef + 4, hb + 20, 16, hipMemcpyHostToDevice, s) == hipSuccess ? 0 : -3);
    C(caxpy_dev(P64, coef + 4, 0, 1.0, v, sv, n, 1, s));
    C(wilson_soa(g, P64, Us, P64, m, sv, t, 1, s));
    C(dot_norm(R, P64, t, sv, n, 1, dsc, 4, s));
    RD();
    double tt = hb[2];
    om = tt > 0 ? H{hb[0] / tt, hb[1] / tt} : H{0, 0};
    // x += al p + om s ; r = s - om t
    hb[24] = al.re; hb[25] = al.im; hb[26] = om.re; hb[27] = om.im; hb[28] = -om.re; hb[29] = -om.im;
    C(hipMemcpyAsync(coef + 8, hb + 24, 48, hipMemcpyHostToDevice, s) == hipSuccess ? 0 : -3);
    C(caxpy_dev(P64, coef + 8, 0, 1.0, p, x, n, 1, s));
    C(caxpy_dev(P64, coef + 10, 0, 1.0, sv, x, n, 1, s));
    C(copy(P64, r, P64, sv, n, 1, s));
    C(caxpy_dev(P64, coef + 12, 0, 1.0, t, r, n, 1, s));
    rho = rho1;
    it++;
    C(norm2(R, P64, r, n, 1, dsc, 4, s));
    RD();
    rn = sqrt(hb[0]);
    if (!std::isfinite(rn)) return set_error(WMG_EBREAKDOWN, "BiCGStab breakdown");
    if (om.re == 0 && om.im == 0) break;
  }
  // true residual
  C(wilson_soa(g, P64, Us, P64, m, x, t, 1, s));
  C(csub(P64, b, t, r, n, 1, s));
  C(norm2(R, P64, r, n, 1, dsc, 4, s));
  RD();
  relres = sqrt(hb[0]) / bn;
  C(spinor_from_soa(g, x, xc, 1, s));
  C(hipStreamSynchronize(s) == hipSuccess ? 0 : -3);
#undef C
#undef RD
  if (st) {
    st->outer_iters = it;
    st->fine_matvecs = 2 * it + 1;
    st->fine_matvecs_fp64 = 2 * it + 1;
    st->coarse_iters = 0;
    st->reliable_updates = 0;
    st->converged = relres <= tol;
    st->true_relres = relres;
    st->setup_s = 0;
    st->solve_s = 0;
  }
  return relres <= tol ? 0 : WMG_ENOTCONV;
}

static int bicgstab_geom(const wmg_geom *gg, Geom &g) {
  for (int i = 0; i < 4; i++) {
    if (gg->L[i] <= 0) return set_error(WMG_EINVAL, "bad extent");
    g.L[i] = gg->L[i];
  }
  g.V = (long)g.L[0] * g.L[1] * g.L[2] * g.L[3];
  g.Vs = fine_stride(g.V);
  return 0;
}

extern "C" int bicgstab_solve(const wmg_geom *gg, const double *U, double m, const double *bc, double *xc, double tol,
                              int maxiter, wmg_stats *st) {
  if (!gg || !U || !bc || !xc || !(tol > 0)) return set_error(WMG_EINVAL, "bad argument");
  Geom g;
  if (int e = bicgstab_geom(gg, g)) return e;
  long n = g.Vs * 12;
  hipStream_t s;
  WMG_HIP(hipStreamCreate(&s));
  BiWork w{};
  std::vector<void *> bufs;
  int rc = 0;
  double *hb = nullptr;
  auto alloc = [&](size_t bytes) -> void * {
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    bufs.push_back(p);
    if (hipMemset(p, 0, bytes) != hipSuccess) return nullptr;  // padding sites stay zero
    return p;
  };
  w.Us = alloc(16 * 36 * (size_t)g.Vs);
  double2 **vecs[8] = {&w.x, &w.b, &w.r, &w.rh, &w.p, &w.v, &w.sv, &w.t};
  bool ok = w.Us != nullptr;
  for (auto q : vecs) ok = ok && (*q = (double2 *)alloc(16 * n)) != nullptr;
  ok = ok && (w.dsc = (double *)alloc(sizeof(double) * 64)) != nullptr;
  if (!ok) rc = set_error(WMG_ENOMEM, "bicgstab allocation");
  else if (hipHostMalloc((void **)&hb, sizeof(double) * 64) != hipSuccess) rc = set_error(WMG_ENOMEM, "pinned");
  else if (!(rc = red_init(w.R, 1))) rc = bicgstab_run(g, U, m, bc, xc, tol, maxiter, st, s, w, hb);
  red_free(w.R);
  for (void *q : bufs) (void)hipFree(q);
  if (hb) (void)hipHostFree(hb);
  (void)hipStreamDestroy(s);
  return rc;
}

// ------------------------------------------------------------ no allocation
// The same solve for callers that cannot allocate device memory: every work
// buffer lives in this fixed device array (one copy per GPU, held until the
// process ends).  Host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[WMG_NOALLOC_SCRATCH_BYTES];

static constexpr int NOALLOC_MAX_DEV = 64;
static std::mutex scratch_mu;
static void *scratch_dev[NOALLOC_MAX_DEV];

static int scratch_ptr(void **out) {
  int dev = 0;
  WMG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEV) return set_error(WMG_EINVAL, "device %d beyond %d", dev, NOALLOC_MAX_DEV);
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (!scratch_dev[dev]) {
    void *ptr = nullptr;
    WMG_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    scratch_dev[dev] = ptr;
  }
  *out = scratch_dev[dev];
  return 0;
}

// bytes of the work buffers for a fine stride Vs, each region 256-aligned
static size_t noalloc_bytes(long Vs, size_t off[11]) {
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  size_t o = 0;
  off[0] = o; o += up(16 * 36 * (size_t)Vs);                         // links
  for (int i = 0; i < 8; i++) { off[1 + i] = o; o += up(16 * 12 * (size_t)Vs); }  // vectors
  off[9] = o; o += up(sizeof(double) * 64);                          // scalars
  off[10] = o; o += up(red_bytes(1));                                // reduction partials
  return o;
}

extern "C" int bicgstab_solve_noalloc(const wmg_geom *gg, const double *U, double m, const double *bc, double *xc,
                                      double tol, int maxiter, wmg_stats *st, void *hip_stream) {
  if (!gg || !U || !bc || !xc || !(tol > 0)) return set_error(WMG_EINVAL, "bad argument");
  Geom g;
  if (int e = bicgstab_geom(gg, g)) return e;
  size_t off[11];
  const size_t need = noalloc_bytes(g.Vs, off);
  if (need > (size_t)WMG_NOALLOC_SCRATCH_BYTES)
    return set_error(WMG_EINVAL, "bicgstab_solve_noalloc: %ld sites need %zu bytes of scratch, the fixed maximum is %zu",
                     g.V, need, (size_t)WMG_NOALLOC_SCRATCH_BYTES);
  void *base = nullptr;
  if (int e = scratch_ptr(&base)) return e;
  hipStream_t s = (hipStream_t)hip_stream;
  unsigned char *b0 = (unsigned char *)base;
  BiWork w{};
  w.Us = b0 + off[0];
  double2 **vecs[8] = {&w.x, &w.b, &w.r, &w.rh, &w.p, &w.v, &w.sv, &w.t};
  for (int i = 0; i < 8; i++) *vecs[i] = (double2 *)(b0 + off[1 + i]);
  w.dsc = (double *)(b0 + off[9]);
  red_attach(w.R, 1, (double *)(b0 + off[10]));
  // the array keeps the previous call's contents: clear every vector (their
  // padding sites must read zero) and the scalars with a fill kernel
  const long n = g.Vs * 12;
  for (int i = 0; i < 8; i++)
    if (int e = zero(P64, *vecs[i], n, 1, s)) return e;
  if (int e = zero(P64, w.dsc, 32, 1, s)) return e;
  double hb[64] = {0};
  return bicgstab_run(g, U, m, bc, xc, tol, maxiter, st, s, w, hb);
}
