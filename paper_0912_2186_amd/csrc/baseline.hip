// Unpreconditioned BiCGStab on the Wilson operator: the unigrid Krylov
// baseline against which the multigrid solve is compared (the paper compares
// MG with unigrid CG-type solvers in Fig. 2-3).  FP64, one right-hand side,
// internal SoA layouts; scalars are read back to the host every iteration.
#include <cmath>
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

extern "C" int bicgstab_solve(const wmg_geom *gg, const double *U, double m, const double *bc, double *xc, double tol,
                              int maxiter, wmg_stats *st) {
  if (!gg || !U || !bc || !xc || !(tol > 0)) return set_error(WMG_EINVAL, "bad argument");
  Geom g;
  for (int i = 0; i < 4; i++) {
    if (gg->L[i] <= 0) return set_error(WMG_EINVAL, "bad extent");
    g.L[i] = gg->L[i];
  }
  g.V = (long)g.L[0] * g.L[1] * g.L[2] * g.L[3];
  g.Vs = fine_stride(g.V);
  long n = g.Vs * 12;
  hipStream_t s;
  WMG_HIP(hipStreamCreate(&s));
  Reducer R{};
  std::vector<void *> bufs;
  int rc = 0;
  double *dsc = nullptr, *hb = nullptr;
  auto alloc = [&](size_t bytes) -> void * {
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    bufs.push_back(p);
    if (hipMemset(p, 0, bytes) != hipSuccess) return nullptr;  // padding sites stay zero
    return p;
  };
  void *Us = alloc(16 * 36 * (size_t)g.Vs);
  double2 *x = (double2 *)alloc(16 * n), *b = (double2 *)alloc(16 * n), *r = (double2 *)alloc(16 * n),
          *rh = (double2 *)alloc(16 * n), *p = (double2 *)alloc(16 * n), *v = (double2 *)alloc(16 * n),
          *sv = (double2 *)alloc(16 * n), *t = (double2 *)alloc(16 * n);
  dsc = (double *)alloc(sizeof(double) * 64);
  int it = 0;
  double relres = 0;
  auto t0 = hipEvent_t{};
  (void)t0;
  if (!Us || !t || !dsc) { rc = set_error(WMG_ENOMEM, "bicgstab allocation"); goto done; }
  if (hipHostMalloc((void **)&hb, sizeof(double) * 64) != hipSuccess) { rc = set_error(WMG_ENOMEM, "pinned"); goto done; }
  if ((rc = red_init(R, 1))) goto done;
#define C(x)            \
  do {                  \
    rc = (x);           \
    if (rc) goto done;  \
  } while (0)
#define RD(k)                                                                                      \
  do {                                                                                             \
    if (hipMemcpyAsync(hb, dsc, sizeof(double) * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||    \
        hipStreamSynchronize(s) != hipSuccess) {                                                   \
      rc = set_error(WMG_EHIP, "readback");                                                        \
      goto done;                                                                                   \
    }                                                                                              \
  } while (0)
  {
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
      // p = r + be (p - om v); every coefficient gets its own pinned and
      // device slot, since the uploads are asynchronous
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
      if (!std::isfinite(rn)) { rc = set_error(WMG_EBREAKDOWN, "BiCGStab breakdown"); goto done; }
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
    rc = relres <= tol ? 0 : WMG_ENOTCONV;
  }
done:
#undef C
#undef RD
  red_free(R);
  for (void *q : bufs) (void)hipFree(q);
  if (hb) (void)hipHostFree(hb);
  (void)hipStreamDestroy(s);
  return rc;
}
