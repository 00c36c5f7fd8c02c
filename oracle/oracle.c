/*
 * Plain FP64 CPU oracle for adaptive-multigrid GCR on the Wilson-Dirac
 * operator (Babich et al., "The role of multigrid algorithms for LQCD",
 * arXiv:0912.2186).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call, link or
 * load this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header, table or helper with the
 * HIP library: it is a second, independent, deliberately slow statement of
 * what the method computes, in double precision, with plain loops.
 *
 * Conventions (the paper fixes none of them, see Sec. 2, Eq. 2.2):
 *   site index   s = x + Lx*(y + Ly*(z + Lz*t)), mu = 0..3 <-> x,y,z,t
 *   gauge field  U[s][mu][a][b]: link from s to s+mu, row a, column b
 *   fine spinor  psi[s][spin*3 + colour]  (12 complex per site)
 *   gamma basis  chiral: gamma_k = [[0,-i sigma_k],[i sigma_k,0]],
 *                gamma_4 = [[0,1],[1,0]], gamma_5 = diag(1,1,-1,-1)
 *   boundaries   periodic in all four directions
 *   chirality    + = first half of the per-site components, - = second half
 *                (spins 0,1 / 2,3 on the fine lattice; sigma_3 = +1 / -1 on
 *                coarse lattices, whose dof are ordered (chi, alpha))
 *   coarse links Y[xh][d][row][col], d = 0 local (X), 1+mu forward
 *                (to xh+mu), 5+mu backward (to xh-mu)
 *   null vectors / prolongator P[alpha][s][dof]; column (xh, alpha, chi) is
 *                P[alpha] restricted to block xh and chirality chi
 *
 * Parity pins: every function here is checked by tests against closed forms,
 * invariants, brute-force dense linear algebra or library routines (see the
 * oracle tests): the cycle against the dense coarse-grid correction and its
 * smoothed and three-level (V, W) forms, the adaptive setup against the
 * near-null space of a dense singular value decomposition.  The setup's
 * vectors themselves are random and iterative: no two correct setups agree
 * vector by vector, so only these properties are pinned.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* ---------------------------------------------------------------------- */
/* gamma matrices (chiral, Hermitian, Euclidean); Eq. 2.2 leaves the basis  */
/* open.                                                                    */
/* ---------------------------------------------------------------------- */
static const cplx GAM[4][4][4] = {
    /* gamma_1 */
    {{0, 0, 0, CMPLX(0, -1)}, {0, 0, CMPLX(0, -1), 0}, {0, CMPLX(0, 1), 0, 0}, {CMPLX(0, 1), 0, 0, 0}},
    /* gamma_2 */
    {{0, 0, 0, -1}, {0, 0, 1, 0}, {0, 1, 0, 0}, {-1, 0, 0, 0}},
    /* gamma_3 */
    {{0, 0, CMPLX(0, -1), 0}, {0, 0, 0, CMPLX(0, 1)}, {CMPLX(0, 1), 0, 0, 0}, {0, CMPLX(0, -1), 0, 0}},
    /* gamma_4 */
    {{0, 0, 1, 0}, {0, 0, 0, 1}, {1, 0, 0, 0}, {0, 1, 0, 0}},
};

void orc_gamma(int mu, double *out /* 4x4 complex interleaved */)
{
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) {
            out[2 * (4 * i + j)] = creal(GAM[mu][i][j]);
            out[2 * (4 * i + j) + 1] = cimag(GAM[mu][i][j]);
        }
}

/* ---------------------------------------------------------------------- */
/* lattice helpers                                                          */
/* ---------------------------------------------------------------------- */
static long vol(const int L[4]) { return (long)L[0] * L[1] * L[2] * L[3]; }

static void coords(const int L[4], long s, int x[4])
{
    for (int mu = 0; mu < 4; mu++) {
        x[mu] = (int)(s % L[mu]);
        s /= L[mu];
    }
}

static long idx(const int L[4], const int x[4])
{
    return x[0] + (long)L[0] * (x[1] + (long)L[1] * (x[2] + (long)L[2] * x[3]));
}

static long nbr(const int L[4], long s, int mu, int sign)
{
    int x[4];
    coords(L, s, x);
    x[mu] = (x[mu] + sign + L[mu]) % L[mu];
    return idx(L, x);
}

/* ---------------------------------------------------------------------- */
/* operators: level 0 = Wilson (Eq. 2.2), level >= 1 = coarse stencil        */
/* ---------------------------------------------------------------------- */
typedef struct {
    int L[4];
    long nsite;
    int dof;        /* complex components per site */
    int kind;       /* 0 Wilson, 1 coarse */
    const cplx *U;  /* Wilson links */
    double m;       /* Wilson mass */
    const cplx *Y;  /* coarse links [nsite][9][dof][dof] */
} orc_op;

/* out_s += hop of direction (mu, sign) of the Wilson operator at site s:
 *   forward : ((gamma_mu - 1)/2) (x) U_mu(x)          psi(x + mu)
 *   backward: -((gamma_mu + 1)/2) (x) U_mu(x - mu)^dag psi(x - mu)
 * This is Eq. 2.2 with the hopping terms placed so that the operator is
 * gauge covariant (the printed Kronecker deltas are read as x+mu = y for the
 * U term and x - mu = y for the U^dag term). */
static void wilson_hop_add(const orc_op *A, long s, int mu, int sign, const cplx *in, cplx *o)
{
    long t = nbr(A->L, s, mu, sign);
    const cplx *ps = in + 12 * t;
    cplx uv[4][3];
    if (sign > 0) {
        const cplx *u = A->U + 9 * (4 * s + mu);
        for (int sp = 0; sp < 4; sp++)
            for (int a = 0; a < 3; a++) {
                cplx acc = 0;
                for (int b = 0; b < 3; b++) acc += u[3 * a + b] * ps[3 * sp + b];
                uv[sp][a] = acc;
            }
    } else {
        const cplx *u = A->U + 9 * (4 * t + mu);
        for (int sp = 0; sp < 4; sp++)
            for (int a = 0; a < 3; a++) {
                cplx acc = 0;
                for (int b = 0; b < 3; b++) acc += conj(u[3 * b + a]) * ps[3 * sp + b];
                uv[sp][a] = acc;
            }
    }
    for (int i = 0; i < 4; i++)
        for (int a = 0; a < 3; a++) {
            cplx acc = 0;
            for (int j = 0; j < 4; j++) {
                cplx g = GAM[mu][i][j] - (i == j ? 1.0 : 0.0); /* gamma - 1 */
                if (sign < 0) g = -(GAM[mu][i][j] + (i == j ? 1.0 : 0.0)); /* -(gamma + 1) */
                acc += 0.5 * g * uv[j][a];
            }
            o[3 * i + a] += acc;
        }
}

static void coarse_hop_add(const orc_op *A, long s, int mu, int sign, const cplx *in, cplx *o)
{
    int n = A->dof;
    long t = nbr(A->L, s, mu, sign);
    const cplx *y = A->Y + ((size_t)s * 9 + (sign > 0 ? 1 + mu : 5 + mu)) * n * n;
    const cplx *v = in + (size_t)n * t;
    for (int r = 0; r < n; r++) {
        cplx acc = 0;
        for (int c = 0; c < n; c++) acc += y[r * n + c] * v[c];
        o[r] += acc;
    }
}

static void op_hop_add(const orc_op *A, long s, int mu, int sign, const cplx *in, cplx *o)
{
    if (A->kind == 0) wilson_hop_add(A, s, mu, sign, in, o);
    else coarse_hop_add(A, s, mu, sign, in, o);
}

static void op_diag_add(const orc_op *A, long s, const cplx *in, cplx *o)
{
    int n = A->dof;
    if (A->kind == 0) {
        for (int c = 0; c < 12; c++) o[c] += (4.0 + A->m) * in[12 * s + c];
    } else {
        const cplx *x = A->Y + (size_t)s * 9 * n * n;
        for (int r = 0; r < n; r++) {
            cplx acc = 0;
            for (int c = 0; c < n; c++) acc += x[r * n + c] * in[(size_t)n * s + c];
            o[r] += acc;
        }
    }
}

/* full operator apply: out = A in */
static void op_apply(const orc_op *A, const cplx *in, cplx *out)
{
    int n = A->dof;
#pragma omp parallel for schedule(static)
    for (long s = 0; s < A->nsite; s++) {
        cplx *o = out + (size_t)n * s;
        for (int c = 0; c < n; c++) o[c] = 0;
        op_diag_add(A, s, in, o);
        for (int mu = 0; mu < 4; mu++) {
            op_hop_add(A, s, mu, +1, in, o);
            op_hop_add(A, s, mu, -1, in, o);
        }
    }
}

/* adjoint of the coarse stencil, written from its definition:
 *   (A^dag v)(x) = X(x)^dag v(x) + sum_mu [ Y_{+mu}(x-mu)^dag v(x-mu)
 *                                         + Y_{-mu}(x+mu)^dag v(x+mu) ] */
static void coarse_apply_dag(const orc_op *A, const cplx *in, cplx *out)
{
    int n = A->dof;
#pragma omp parallel for schedule(static)
    for (long s = 0; s < A->nsite; s++) {
        cplx *o = out + (size_t)n * s;
        for (int r = 0; r < n; r++) o[r] = 0;
        for (int d = 0; d < 9; d++) {
            long src;
            int blk;
            if (d == 0) { src = s; blk = 0; }
            else if (d <= 4) { src = nbr(A->L, s, d - 1, -1); blk = d; }      /* Y_{+mu}(x-mu) */
            else { src = nbr(A->L, s, d - 5, +1); blk = d; }                 /* Y_{-mu}(x+mu) */
            const cplx *y = A->Y + ((size_t)src * 9 + blk) * n * n;
            const cplx *v = in + (size_t)n * src;
            for (int r = 0; r < n; r++) {
                cplx acc = 0;
                for (int c = 0; c < n; c++) acc += conj(y[c * n + r]) * v[c];
                o[r] += acc;
            }
        }
    }
}

/* ---------------------------------------------------------------------- */
/* vector algebra (plain)                                                   */
/* ---------------------------------------------------------------------- */
static cplx vdot(long n, const cplx *a, const cplx *b) /* sum conj(a) b */
{
    double re = 0, im = 0;
#pragma omp parallel for reduction(+ : re, im) schedule(static)
    for (long i = 0; i < n; i++) {
        cplx t = conj(a[i]) * b[i];
        re += creal(t);
        im += cimag(t);
    }
    return CMPLX(re, im);
}

static double vnorm2(long n, const cplx *a)
{
    double r = 0;
#pragma omp parallel for reduction(+ : r) schedule(static)
    for (long i = 0; i < n; i++) r += creal(a[i]) * creal(a[i]) + cimag(a[i]) * cimag(a[i]);
    return r;
}

static void vaxpy(long n, cplx a, const cplx *x, cplx *y) /* y += a x */
{
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; i++) y[i] += a * x[i];
}

static void vcopy(long n, const cplx *x, cplx *y) { memcpy(y, x, sizeof(cplx) * n); }
static void vzero(long n, cplx *y) { memset(y, 0, sizeof(cplx) * n); }
static cplx *valloc(long n) { return (cplx *)calloc((size_t)(n > 0 ? n : 1), sizeof(cplx)); }

/* ---------------------------------------------------------------------- */
/* red/black (even-odd) decomposition (Sec. 3: MG combined with red/black    */
/* preconditioning).  Sites split by parity (x+y+z+t) mod 2, and with that   */
/* D = [[D_ee, D_eo], [D_oe, D_oo]]: the only site-local term of Eq. 2.2 is  */
/* the (4+m) diagonal, so D_ee = D_oo = (4+m) 1, and D_eo, D_oe are the      */
/* hopping terms between the sublattices.  With x_o eliminated, D x = b      */
/* becomes the Schur complement system on the even sites                    */
/*   S x_e = b_e - D_eo D_oo^-1 b_o,   S = D_ee - D_eo D_oo^-1 D_oe,         */
/* and x_o = D_oo^-1 (b_o - D_oe x_e).  Vectors here are full length; the    */
/* components of sites outside the parity a function works on are ignored  */
/* on input and zero on output.                                              */
/* ---------------------------------------------------------------------- */
int orc_parity(const int L[4], long s)
{
    int x[4];
    coords(L, s, x);
    return (x[0] + x[1] + x[2] + x[3]) & 1;
}

/* out = D_{par, 1-par} in: the hopping terms of Eq. 2.2 at the sites of
 * parity par, reading in at the sites of the other parity */
void orc_wilson_hop_parity(const int L[4], const double *U, double m, const double *ind, double *outd, int par)
{
    orc_op A = {{L[0], L[1], L[2], L[3]}, vol(L), 12, 0, (const cplx *)U, m, NULL};
    const cplx *in = (const cplx *)ind;
    cplx *out = (cplx *)outd;
    long V = A.nsite;
    cplx *src = valloc(V * 12);
    for (long s = 0; s < V; s++)
        if (orc_parity(L, s) != par) memcpy(src + 12 * s, in + 12 * s, sizeof(cplx) * 12);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; s++) {
        cplx *o = out + 12 * s;
        for (int c = 0; c < 12; c++) o[c] = 0;
        if (orc_parity(L, s) != par) continue;
        for (int mu = 0; mu < 4; mu++) {
            wilson_hop_add(&A, s, mu, +1, src, o);
            wilson_hop_add(&A, s, mu, -1, src, o);
        }
    }
    free(src);
}

/* out_e = S in_e = (4+m) in_e - D_eo (D_oe in_e) / (4+m) */
void orc_schur_apply(const int L[4], const double *U, double m, const double *ind, double *outd)
{
    long V = vol(L), n = V * 12;
    const cplx *in = (const cplx *)ind;
    cplx *out = (cplx *)outd;
    cplx *t = valloc(n), *u = valloc(n);
    orc_wilson_hop_parity(L, U, m, ind, (double *)t, 1);   /* t_o = D_oe in_e */
    for (long i = 0; i < n; i++) t[i] /= (4.0 + m);         /* D_oo^-1 */
    orc_wilson_hop_parity(L, U, m, (const double *)t, (double *)u, 0); /* u_e = D_eo t_o */
    for (long s = 0; s < V; s++)
        for (int c = 0; c < 12; c++)
            out[12 * s + c] = orc_parity(L, s) == 0 ? (4.0 + m) * in[12 * s + c] - u[12 * s + c] : 0;
    free(t);
    free(u);
}

/* ---------------------------------------------------------------------- */
/* public single-operator entry points                                      */
/* ---------------------------------------------------------------------- */
/* Eq. 2.2: out = D(U) in (full operator including the (4+m) diagonal). */
void orc_wilson(const int L[4], const double *U, double m, const double *in, double *out)
{
    orc_op A = {{L[0], L[1], L[2], L[3]}, vol(L), 12, 0, (const cplx *)U, m, NULL};
    op_apply(&A, (const cplx *)in, (cplx *)out);
}

void orc_coarse_apply(const int L[4], int dof, const double *Y, const double *in, double *out, int dagger)
{
    orc_op A = {{L[0], L[1], L[2], L[3]}, vol(L), dof, 1, NULL, 0, (const cplx *)Y};
    if (dagger) coarse_apply_dag(&A, (const cplx *)in, (cplx *)out);
    else op_apply(&A, (const cplx *)in, (cplx *)out);
}

/* ---------------------------------------------------------------------- */
/* blocking: Eq. 2.4 theta functions, Eq. 2.7 block orthonormalisation,     */
/* chirality split of Sec. 3 (sigma_3 P = P gamma_5)                        */
/* ---------------------------------------------------------------------- */
static void coarse_dims(const int L[4], const int b[4], int Lc[4])
{
    for (int mu = 0; mu < 4; mu++) Lc[mu] = L[mu] / b[mu];
}

static long block_of(const int L[4], const int b[4], long s)
{
    int x[4], xc[4], Lc[4];
    coords(L, s, x);
    coarse_dims(L, b, Lc);
    for (int mu = 0; mu < 4; mu++) xc[mu] = x[mu] / b[mu];
    return idx(Lc, xc);
}

/* list the fine sites of coarse site xh in a fixed order (x fastest) */
static void block_sites(const int L[4], const int b[4], long xh, long *sites)
{
    int Lc[4], xc[4], x[4];
    coarse_dims(L, b, Lc);
    coords(Lc, xh, xc);
    long k = 0;
    for (int t = 0; t < b[3]; t++)
        for (int z = 0; z < b[2]; z++)
            for (int y = 0; y < b[1]; y++)
                for (int xx = 0; xx < b[0]; xx++) {
                    x[0] = xc[0] * b[0] + xx;
                    x[1] = xc[1] * b[1] + y;
                    x[2] = xc[2] * b[2] + z;
                    x[3] = xc[3] * b[3] + t;
                    sites[k++] = idx(L, x);
                }
}

/* Eq. 2.7: for every block xh and part chi of the per-site components,
 * replace the restrictions theta_xh(x) Pi_chi psi^(alpha) (alpha = 0..nv-1,
 * in order) by an orthonormal basis of their span: modified Gram-Schmidt
 * run twice, unit norms, diag(R) > 0.  The components split into ns equal
 * parts: ns = 2 the chiralities of Sec. 3 (spins 0,1 / 2,3 on the fine
 * lattice), ns = 4 the four Dirac spins (the full spin structure the
 * paper's Sec. 3 exposes on the coarse blocks as a variant).  Returns 0, or
 * -4 on rank breakdown. */
int orc_block_orthonormalize_ns(const int L[4], int dof, const int b[4], int nv, int ns, const double *vecs_in,
                                double *P_out)
{
    long V = vol(L);
    int Lc[4];
    coarse_dims(L, b, Lc);
    long Vc = vol(Lc), bs = (long)b[0] * b[1] * b[2] * b[3];
    int h = dof / ns;
    const cplx *vin = (const cplx *)vecs_in;
    cplx *P = (cplx *)P_out;
    if (P != vin) memcpy(P, vin, sizeof(cplx) * (size_t)nv * V * dof);
    int fail = 0;
#pragma omp parallel for schedule(dynamic) reduction(| : fail)
    for (long q = 0; q < ns * Vc; q++) {
        long xh = q / ns;
        int chi = (int)(q % ns);
        long *sites = malloc(sizeof(long) * bs);
        block_sites(L, b, xh, sites);
        long n = bs * h;
        cplx *w = malloc(sizeof(cplx) * n * nv);
        for (int a = 0; a < nv; a++)
            for (long k = 0; k < bs; k++)
                for (int c = 0; c < h; c++)
                    w[a * n + k * h + c] = P[((size_t)a * V + sites[k]) * dof + chi * h + c];
        for (int a = 0; a < nv; a++) {
            cplx *va = w + a * n;
            double n0 = 0;
            for (long i = 0; i < n; i++) n0 += creal(conj(va[i]) * va[i]);
            for (int pass = 0; pass < 2; pass++)
                for (int j = 0; j < a; j++) {
                    cplx *qj = w + j * n, p = 0;
                    for (long i = 0; i < n; i++) p += conj(qj[i]) * va[i];
                    for (long i = 0; i < n; i++) va[i] -= p * qj[i];
                }
            double nn = 0;
            for (long i = 0; i < n; i++) nn += creal(conj(va[i]) * va[i]);
            if (!(nn > 1e-24 * n0) || n0 == 0) { fail = 1; nn = 1; }
            double inv = 1.0 / sqrt(nn);
            for (long i = 0; i < n; i++) va[i] *= inv;
        }
        for (int a = 0; a < nv; a++)
            for (long k = 0; k < bs; k++)
                for (int c = 0; c < h; c++)
                    P[((size_t)a * V + sites[k]) * dof + chi * h + c] = w[a * n + k * h + c];
        free(w);
        free(sites);
    }
    return fail ? -4 : 0;
}

int orc_block_orthonormalize(const int L[4], int dof, const int b[4], int nv, const double *vecs_in,
                             double *P_out)
{
    return orc_block_orthonormalize_ns(L, dof, b, nv, 2, vecs_in, P_out);
}

/* r_hat = P^dag r  (coarse dof index chi*nv + alpha, chi one of ns parts) */
void orc_restrict_ns(const int L[4], int dof, const int b[4], int nv, int ns, const double *Pd, const double *fine,
                     double *coarse)
{
    long V = vol(L);
    int Lc[4];
    coarse_dims(L, b, Lc);
    long Vc = vol(Lc), bs = (long)b[0] * b[1] * b[2] * b[3];
    int h = dof / ns, nc = ns * nv;
    const cplx *P = (const cplx *)Pd, *f = (const cplx *)fine;
    cplx *c = (cplx *)coarse;
#pragma omp parallel for schedule(static)
    for (long xh = 0; xh < Vc; xh++) {
        long *sites = malloc(sizeof(long) * bs);
        block_sites(L, b, xh, sites);
        for (int chi = 0; chi < ns; chi++)
            for (int a = 0; a < nv; a++) {
                cplx acc = 0;
                for (long k = 0; k < bs; k++)
                    for (int cc = chi * h; cc < (chi + 1) * h; cc++)
                        acc += conj(P[((size_t)a * V + sites[k]) * dof + cc]) * f[(size_t)sites[k] * dof + cc];
                c[xh * nc + chi * nv + a] = acc;
            }
        free(sites);
    }
}

void orc_restrict(const int L[4], int dof, const int b[4], int nv, const double *Pd, const double *fine,
                  double *coarse)
{
    orc_restrict_ns(L, dof, b, nv, 2, Pd, fine, coarse);
}

/* e = P e_hat   (Eq. 2.3) */
void orc_prolong_ns(const int L[4], int dof, const int b[4], int nv, int ns, const double *Pd, const double *coarse,
                    double *fine)
{
    long V = vol(L);
    int h = dof / ns, nc = ns * nv;
    const cplx *P = (const cplx *)Pd, *c = (const cplx *)coarse;
    cplx *f = (cplx *)fine;
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; s++) {
        long xh = block_of(L, b, s);
        for (int cc = 0; cc < dof; cc++) {
            int chi = cc / h;
            cplx acc = 0;
            for (int a = 0; a < nv; a++) acc += P[((size_t)a * V + s) * dof + cc] * c[xh * nc + chi * nv + a];
            f[(size_t)s * dof + cc] = acc;
        }
    }
}

void orc_prolong(const int L[4], int dof, const int b[4], int nv, const double *Pd, const double *coarse,
                 double *fine)
{
    orc_prolong_ns(L, dof, b, nv, 2, Pd, coarse, fine);
}

/* Galerkin coarse operator D_hat = P^dag D P (Sec. 2), stored as a 9-point
 * stencil.  For every coarse column (chi_c, alpha) the fine vector
 * v = Pi_chi_c P[alpha] (all blocks at once) is hit by D split by hop class:
 * class 0 = diagonal + hops that stay inside the target site's block,
 * class 1+mu / 5+mu = hops in +mu / -mu that cross the block face.  Each
 * class result is restricted on the target block, giving column entries of
 * X (class 0) and Y_{+-mu}.  Keeping classes apart by hop direction keeps
 * the forward and backward links apart even where the coarse extent is 1 or
 * 2 and both neighbours are the same coarse site. */
static void coarse_build(const orc_op *A, const int b[4], int nv, int ns, const cplx *P, cplx *Y)
{
    const int *L = A->L;
    long V = A->nsite;
    int dof = A->dof, h = dof / ns, nd = ns * nv;
    int Lc[4];
    coarse_dims(L, b, Lc);
    long Vc = vol(Lc), bs = (long)b[0] * b[1] * b[2] * b[3];
    memset(Y, 0, sizeof(cplx) * (size_t)Vc * 9 * nd * nd);
    cplx *v = valloc(V * dof);
    for (int col = 0; col < nd; col++) {
        int chic = col / nv, al = col % nv;
        vzero(V * dof, v);
        for (long s = 0; s < V; s++)
            for (int c = chic * h; c < (chic + 1) * h; c++) v[(size_t)s * dof + c] = P[((size_t)al * V + s) * dof + c];
#pragma omp parallel for schedule(dynamic)
        for (long xh = 0; xh < Vc; xh++) {
            long *sites = malloc(sizeof(long) * bs);
            cplx *w = malloc(sizeof(cplx) * 9 * dof);
            cplx *tmp = malloc(sizeof(cplx) * dof);
            block_sites(L, b, xh, sites);
            for (long k = 0; k < bs; k++) {
                long s = sites[k];
                int x[4];
                coords(L, s, x);
                memset(w, 0, sizeof(cplx) * 9 * dof);
                op_diag_add(A, s, v, w);
                for (int mu = 0; mu < 4; mu++)
                    for (int sg = -1; sg <= 1; sg += 2) {
                        int cross = sg > 0 ? (x[mu] % b[mu] == b[mu] - 1) : (x[mu] % b[mu] == 0);
                        int cls = cross ? (sg > 0 ? 1 + mu : 5 + mu) : 0;
                        memset(tmp, 0, sizeof(cplx) * dof);
                        op_hop_add(A, s, mu, sg, v, tmp);
                        for (int c = 0; c < dof; c++) w[cls * dof + c] += tmp[c];
                    }
                for (int d = 0; d < 9; d++)
                    for (int row = 0; row < nd; row++) {
                        int chir = row / nv, be = row % nv;
                        cplx acc = 0;
                        for (int c = chir * h; c < (chir + 1) * h; c++)
                            acc += conj(P[((size_t)be * V + s) * dof + c]) * w[d * dof + c];
                        Y[(((size_t)xh * 9 + d) * nd + row) * nd + col] += acc;
                    }
            }
            free(tmp);
            free(w);
            free(sites);
        }
    }
    free(v);
}

/* public wrapper: level operator given by (kind, U, m) or (kind, Y); ns
 * parts per site (2 chiralities, or 4 spins on the fine level) */
void orc_coarse_build_ns(const int L[4], int kind, int dof, const double *U, double m, const double *Yf,
                         const int b[4], int nv, int ns, const double *P, double *Yc)
{
    orc_op A = {{L[0], L[1], L[2], L[3]}, vol(L), kind == 0 ? 12 : dof, kind, (const cplx *)U, m,
                (const cplx *)Yf};
    coarse_build(&A, b, nv, ns, (const cplx *)P, (cplx *)Yc);
}

void orc_coarse_build(const int L[4], int kind, int dof, const double *U, double m, const double *Yf,
                      const int b[4], int nv, const double *P, double *Yc)
{
    orc_coarse_build_ns(L, kind, dof, U, m, Yf, b, nv, 2, P, Yc);
}

/* ---------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): counter-based random  */
/* numbers for the setup's random start vectors.                            */
/* ---------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; r++) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* random start vector alpha of level lvl: component (s, c) gets
 * re = int32(w0) * 2^-31, im = int32(w1) * 2^-31 with
 * (w0..w3) = Philox(ctr = (c, s, alpha, lvl), key = (seed lo, seed hi)). */
void orc_start_vector(long nsite, int dof, uint64_t seed, int lvl, int alpha, double *out)
{
    cplx *o = (cplx *)out;
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
#pragma omp parallel for schedule(static)
    for (long s = 0; s < nsite; s++)
        for (int c = 0; c < dof; c++) {
            uint32_t ctr[4] = {(uint32_t)c, (uint32_t)s, (uint32_t)alpha, (uint32_t)lvl}, w[4];
            orc_philox4x32_10(ctr, key, w);
            o[(size_t)s * dof + c] = CMPLX((double)(int32_t)w[0] * 0x1p-31, (double)(int32_t)w[1] * 0x1p-31);
        }
}

/* ---------------------------------------------------------------------- */
/* multigrid hierarchy                                                      */
/* ---------------------------------------------------------------------- */
typedef struct {
    int nlevels;      /* 2 or 3 */
    int block[2][4];  /* blocking of level l -> l+1 */
    int nv[2];        /* null vectors per level */
    int setup_iters;  /* GCR iterations per null vector (adaptive setup) */
    int post_smooth;  /* MR post-smoothing steps */
    int gcr_restart;  /* outer GCR restart length */
    int wcycle;       /* 1 = W-cycle, 0 = V-cycle */
    double coarse_tol;
    int coarse_maxiter;
    int maxiter;
    uint64_t seed;
    int eo_smoother;  /* 1: fine-level post-smoother on the red/black Schur complement */
    int spin_parts;   /* parts per fine site in the blocking of level 0: 2 (chirality) or 4 (spin) */
} orc_mg_params;

typedef struct {
    long outer_iters;
    long fine_matvecs;
    long coarse_iters;  /* CGNR iterations, all coarse solves */
    long restarts;
    int converged;
    double true_relres;
} orc_stats;

typedef struct {
    orc_op op;
    cplx *Ybuf;  /* owned coarse links */
    cplx *P;     /* [nv][nsite][dof] prolongator to the next level */
    cplx *vecs;  /* [nv][nsite][dof] adapted null vectors before block
                    orthonormalisation (kept after the setup for inspection) */
    int nv;
    int b[4];
    long n;      /* nsite * dof */
} orc_lvl;

typedef struct {
    orc_mg_params p;
    int nl;
    orc_lvl lv[3];
    cplx *U;
    double m;
} orc_mg;

/* parts per site of the blocking of level l: chirality (2), or the four
 * spins on the fine level when spin_parts = 4 */
static int lvl_parts(const orc_mg *g, int l) { return l == 0 && g->p.spin_parts == 4 ? 4 : 2; }

static void lvl_apply(orc_mg *g, int l, const cplx *in, cplx *out, orc_stats *st)
{
    op_apply(&g->lv[l].op, in, out);
    if (l == 0 && st) st->fine_matvecs++;
}

/* MR smoother (reading of the unnamed fine-level smoother of Sec. 2/3):
 * nsteps minimal-residual steps on A e = r starting from e. */
static void mr_smooth(orc_mg *g, int l, const cplx *r, cplx *e, int nsteps, orc_stats *st)
{
    long n = g->lv[l].n;
    cplx *s = valloc(n), *q = valloc(n);
    lvl_apply(g, l, e, s, st);
    for (long i = 0; i < n; i++) s[i] = r[i] - s[i];
    for (int k = 0; k < nsteps; k++) {
        lvl_apply(g, l, s, q, st);
        double qq = vnorm2(n, q);
        if (qq == 0) break;
        cplx a = vdot(n, q, s) / qq;
        vaxpy(n, a, s, e);
        vaxpy(n, -a, q, s);
    }
    free(s);
    free(q);
}

/* Red/black post-smoother of the fine level (Sec. 3: MG combined with
 * red/black preconditioning; reading: the smoother's minimal-residual steps
 * run on the Schur complement).  With s = r - D e, the correction d solving
 * D d = s is split into sublattices: d_e from nsteps MR steps on
 * S d_e = s_e - D_eo D_oo^-1 s_o starting from 0, and d_o = D_oo^-1
 * (s_o - D_oe d_e) exactly; then e += d. */
static void mr_smooth_schur(orc_mg *g, const cplx *r, cplx *e, int nsteps, orc_stats *st)
{
    const orc_op *A = &g->lv[0].op;
    const double *U = (const double *)g->U;
    double m = A->m;
    long V = A->nsite, n = V * 12;
    cplx *s = valloc(n), *t = valloc(n), *be = valloc(n), *d = valloc(n), *q = valloc(n);
    lvl_apply(g, 0, e, s, st);
    for (long i = 0; i < n; i++) s[i] = r[i] - s[i];
    orc_wilson_hop_parity(A->L, U, m, (const double *)s, (double *)t, 0); /* D_eo s_o */
    for (long x = 0; x < V; x++)
        for (int c = 0; c < 12; c++)
            be[12 * x + c] = orc_parity(A->L, x) ? 0 : s[12 * x + c] - t[12 * x + c] / (4.0 + m);
    /* MR on S d_e = be from d_e = 0: residual be - S d_e lives in be */
    for (int k = 0; k < nsteps; k++) {
        orc_schur_apply(A->L, U, m, (const double *)be, (double *)q);
        if (st) st->fine_matvecs += 1;
        double qq = vnorm2(n, q);
        if (qq == 0) break;
        cplx a = vdot(n, q, be) / qq;
        vaxpy(n, a, be, d);
        vaxpy(n, -a, q, be);
    }
    orc_wilson_hop_parity(A->L, U, m, (const double *)d, (double *)t, 1); /* D_oe d_e */
    for (long x = 0; x < V; x++)
        if (orc_parity(A->L, x))
            for (int c = 0; c < 12; c++) d[12 * x + c] = (s[12 * x + c] - t[12 * x + c]) / (4.0 + m);
    vaxpy(n, 1.0, d, e);
    free(s); free(t); free(be); free(d); free(q);
}

/* CG on the normal equations A^dag A x = A^dag b at the coarsest level
 * (Sec. 3); stops when the true coarse residual |b - A x| <= tol |b|. */
static long cgnr(const orc_op *A, const cplx *b, cplx *x, double tol, int maxiter)
{
    long n = A->nsite * A->dof;
    cplx *r = valloc(n), *s = valloc(n), *p = valloc(n), *u = valloc(n);
    vzero(n, x);
    vcopy(n, b, r);
    double bn = sqrt(vnorm2(n, b));
    long it = 0;
    if (bn == 0) goto done;
    coarse_apply_dag(A, r, s);
    vcopy(n, s, p);
    double ss = vnorm2(n, s);
    while (it < maxiter) {
        op_apply(A, p, u);
        double uu = vnorm2(n, u);
        if (uu == 0) break;
        double a = ss / uu;
        vaxpy(n, a, p, x);
        vaxpy(n, -a, u, r);
        it++;
        if (sqrt(vnorm2(n, r)) <= tol * bn) break;
        coarse_apply_dag(A, r, s);
        double ss1 = vnorm2(n, s);
        double be = ss1 / ss;
        ss = ss1;
        for (long i = 0; i < n; i++) p[i] = s[i] + be * p[i];
    }
done:
    free(r); free(s); free(p); free(u);
    return it;
}

/* one multigrid cycle at level l: e = M_l r (Sec. 2-3):
 * restrict, coarse correction (CGNR at the coarsest level, else recursive
 * V or W cycle), prolong, post-smooth.  No pre-smoothing. */
static void mg_cycle(orc_mg *g, int l, const cplx *r, cplx *e, orc_stats *st)
{
    orc_lvl *F = &g->lv[l], *C = &g->lv[l + 1];
    cplx *rc = valloc(C->n), *ec = valloc(C->n);
    orc_restrict_ns(F->op.L, F->op.dof, F->b, F->nv, lvl_parts(g, l), (const double *)F->P, (const double *)r,
                    (double *)rc);
    if (l + 1 == g->nl - 1) {
        long it = cgnr(&C->op, rc, ec, g->p.coarse_tol, g->p.coarse_maxiter);
        if (st) st->coarse_iters += it;
    } else {
        mg_cycle(g, l + 1, rc, ec, st);
        if (g->p.wcycle) {
            cplx *t = valloc(C->n), *e2 = valloc(C->n);
            lvl_apply(g, l + 1, ec, t, st);
            for (long i = 0; i < C->n; i++) t[i] = rc[i] - t[i];
            mg_cycle(g, l + 1, t, e2, st);
            vaxpy(C->n, 1.0, e2, ec);
            free(t);
            free(e2);
        }
    }
    orc_prolong_ns(F->op.L, F->op.dof, F->b, F->nv, lvl_parts(g, l), (const double *)F->P, (const double *)ec,
                   (double *)e);
    if (l == 0 && g->p.eo_smoother) mr_smooth_schur(g, r, e, g->p.post_smooth, st);
    else mr_smooth(g, l, r, e, g->p.post_smooth, st);
    free(rc);
    free(ec);
}

typedef void (*precond_fn)(orc_mg *g, int l, const cplx *r, cplx *z, orc_stats *st);
typedef void (*apply_fn)(orc_mg *g, int l, const cplx *in, cplx *out, orc_stats *st);

static void pc_cycle(orc_mg *g, int l, const cplx *r, cplx *z, orc_stats *st) { mg_cycle(g, l, r, z, st); }

/* red/black: the Schur complement S on the even sites of level 0 */
static void schur_apply_lvl(orc_mg *g, int l, const cplx *in, cplx *out, orc_stats *st)
{
    (void)l;
    orc_schur_apply(g->lv[0].op.L, (const double *)g->U, g->lv[0].op.m, (const double *)in, (double *)out);
    if (st) st->fine_matvecs += 1; /* two half-lattice hopping applies */
}

/* red/black preconditioner: [D^-1 (r_e, 0)]_e = S^-1 r_e exactly, so the
 * multigrid cycle for D applied to (r_e, 0) and restricted to the even sites
 * approximates S^-1 */
static void pc_cycle_even(orc_mg *g, int l, const cplx *r, cplx *z, orc_stats *st)
{
    const orc_op *A = &g->lv[0].op;
    mg_cycle(g, 0, r, z, st);
    for (long s = 0; s < A->nsite; s++)
        if (orc_parity(A->L, s)) memset(z + 12 * s, 0, sizeof(cplx) * 12);
    (void)l;
}

static void pc_smoother(orc_mg *g, int l, const cplx *r, cplx *z, orc_stats *st)
{
    vzero(g->lv[l].n, z);
    mr_smooth(g, l, r, z, g->p.post_smooth, st);
}

/* flexible restarted GCR (Sec. 3 outer solver).  Each restart cycle keeps
 * the preconditioned directions z_k and the orthonormalised w_k = A z_k -
 * sum beta_jk w_j; at its end the solution update is recovered from the
 * triangular system and the true residual is recomputed. */
static long gcr_op(orc_mg *g, int l, const cplx *b, cplx *x, double tol, int maxiter, precond_fn M, apply_fn A,
                   double bnorm, orc_stats *st);

static long gcr(orc_mg *g, int l, const cplx *b, cplx *x, double tol, int maxiter, precond_fn M, orc_stats *st)
{
    return gcr_op(g, l, b, x, tol, maxiter, M, lvl_apply, -1.0, st);
}

/* the same with operator A; bnorm >= 0 replaces |b| in the stopping test */
static long gcr_op(orc_mg *g, int l, const cplx *b, cplx *x, double tol, int maxiter, precond_fn M, apply_fn A,
                   double bnorm, orc_stats *st)
{
    long n = g->lv[l].n;
    int K = g->p.gcr_restart;
    cplx **z = malloc(sizeof(cplx *) * K), **w = malloc(sizeof(cplx *) * K);
    for (int k = 0; k < K; k++) { z[k] = valloc(n); w[k] = valloc(n); }
    cplx *r = valloc(n), *al = calloc(K, sizeof(cplx)), *be = calloc(K * K, sizeof(cplx)), *cc = calloc(K, sizeof(cplx));
    double *ga = calloc(K, sizeof(double));
    double bn = bnorm >= 0 ? bnorm : sqrt(vnorm2(n, b));
    if (vnorm2(n, x) == 0) {
        vcopy(n, b, r); /* zero initial guess: no operator apply needed */
    } else {
        A(g, l, x, r, st);
        for (long i = 0; i < n; i++) r[i] = b[i] - r[i];
    }
    double rn = sqrt(vnorm2(n, r));
    long it = 0;
    int done = rn <= tol * bn;
    while (!done && it < maxiter) {
        int k = 0;
        while (k < K && it < maxiter) {
            M(g, l, r, z[k], st);
            A(g, l, z[k], w[k], st);
            for (int j = 0; j < k; j++) {
                be[j * K + k] = vdot(n, w[j], w[k]);
                vaxpy(n, -be[j * K + k], w[j], w[k]);
            }
            ga[k] = sqrt(vnorm2(n, w[k]));
            if (ga[k] == 0) { done = 1; break; }
            for (long i = 0; i < n; i++) w[k][i] /= ga[k];
            al[k] = vdot(n, w[k], r);
            vaxpy(n, -al[k], w[k], r);
            k++;
            it++;
            rn = sqrt(vnorm2(n, r));
            if (rn <= tol * bn) break;
        }
        for (int j = k - 1; j >= 0; j--) {
            cplx t = al[j];
            for (int i = j + 1; i < k; i++) t -= be[j * K + i] * cc[i];
            cc[j] = t / ga[j];
        }
        for (int j = 0; j < k; j++) vaxpy(n, cc[j], z[j], x);
        A(g, l, x, r, st);
        for (long i = 0; i < n; i++) r[i] = b[i] - r[i];
        rn = sqrt(vnorm2(n, r));
        if (st) st->restarts++;
        if (rn <= tol * bn) done = 1;
    }
    if (st) {
        st->outer_iters += it;
        st->converged = rn <= tol * bn;
        st->true_relres = bn > 0 ? rn / bn : rn;
    }
    for (int k = 0; k < K; k++) { free(z[k]); free(w[k]); }
    free(z); free(w); free(r); free(al); free(be); free(cc); free(ga);
    return it;
}

static void lvl_set_op(orc_mg *g, int l)
{
    orc_lvl *F = &g->lv[l], *C = &g->lv[l + 1];
    coarse_dims(F->op.L, F->b, C->op.L);
    C->op.nsite = vol(C->op.L);
    C->op.dof = lvl_parts(g, l) * F->nv;
    C->op.kind = 1;
    C->n = C->op.nsite * C->op.dof;
}

/* build P_l from the first k vectors of vecs (block Gram-Schmidt) and the
 * Galerkin coarse operator of level l+1 */
static int build_level(orc_mg *g, int l, const cplx *vecs, int k)
{
    orc_lvl *F = &g->lv[l], *C = &g->lv[l + 1];
    int nv_full = F->nv;
    F->nv = k;
    lvl_set_op(g, l);
    int rc = orc_block_orthonormalize_ns(F->op.L, F->op.dof, F->b, k, lvl_parts(g, l), (const double *)vecs,
                                         (double *)F->P);
    coarse_build(&F->op, F->b, k, lvl_parts(g, l), F->P, C->Ybuf);
    C->op.Y = C->Ybuf;
    if (k != nv_full) { /* trial scheme: remember the size used */ }
    return rc;
}

orc_mg *orc_mg_create(const int L[4], const double *U, double m, const orc_mg_params *p)
{
    orc_mg *g = calloc(1, sizeof(orc_mg));
    g->p = *p;
    g->nl = p->nlevels;
    g->m = m;
    long V = vol(L);
    g->U = malloc(sizeof(cplx) * V * 36);
    memcpy(g->U, U, sizeof(cplx) * V * 36);
    orc_lvl *F = &g->lv[0];
    memcpy(F->op.L, L, sizeof(int) * 4);
    F->op.nsite = V;
    F->op.dof = 12;
    F->op.kind = 0;
    F->op.U = g->U;
    F->op.m = m;
    F->n = V * 12;
    for (int l = 0; l + 1 < g->nl; l++) {
        orc_lvl *A = &g->lv[l], *C = &g->lv[l + 1];
        memcpy(A->b, p->block[l], sizeof(int) * 4);
        A->nv = p->nv[l];
        A->P = valloc((long)A->nv * A->n);
        A->vecs = valloc((long)A->nv * A->n);
        lvl_set_op(g, l);
        C->Ybuf = valloc(C->op.nsite * 9L * C->op.dof * C->op.dof);
        C->op.Y = C->Ybuf;
    }
    return g;
}

void orc_mg_free(orc_mg *g)
{
    if (!g) return;
    for (int l = 0; l < 3; l++) { free(g->lv[l].P); free(g->lv[l].vecs); free(g->lv[l].Ybuf); }
    free(g->U);
    free(g);
}

/* Adaptive setup of level l (Sec. 2, Eq. 2.6): null vectors are found one
 * after the other.  Vector k starts from a Philox random vector and is
 * relaxed on A x = 0 by setup_iters iterations of GCR preconditioned with the
 * trial multigrid scheme built from vectors 0..k-1 (for k = 0 there is no
 * coarse space yet and the preconditioner is the smoother alone), then
 * normalised.  After the last vector the level is built from all of them. */
static int setup_level(orc_mg *g, int l, orc_stats *st)
{
    orc_lvl *F = &g->lv[l];
    int nv = F->nv;
    long n = F->n;
    cplx *vecs = valloc((long)nv * n);
    cplx *zero = valloc(n);
    int save_nl = g->nl, rc = 0;
    g->nl = l + 2; /* trial scheme is two-level: level l and its coarse CGNR */
    for (int k = 0; k < nv; k++) {
        cplx *x = vecs + (size_t)k * n;
        orc_start_vector(F->op.nsite, F->op.dof, g->p.seed, l, k, (double *)x);
        if (k > 0) {
            rc = build_level(g, l, vecs, k);
            if (rc) break;
        }
        gcr(g, l, zero, x, 0.0, g->p.setup_iters, k > 0 ? pc_cycle : pc_smoother, NULL);
        double nx = sqrt(vnorm2(n, x));
        for (long i = 0; i < n; i++) x[i] /= nx;
    }
    F->nv = nv;
    if (!rc) rc = build_level(g, l, vecs, nv);
    g->nl = save_nl;
    memcpy(F->vecs, vecs, sizeof(cplx) * (size_t)nv * n);
    free(vecs);
    free(zero);
    (void)st;
    return rc;
}

int orc_mg_setup(orc_mg *g)
{
    for (int l = 0; l + 1 < g->nl; l++) {
        int rc = setup_level(g, l, NULL);
        if (rc) return rc;
    }
    return 0;
}

/* install given null vectors at level l (and rebuild P_l and level l+1) */
int orc_mg_set_null_vectors(orc_mg *g, int l, const double *vecs)
{
    memcpy(g->lv[l].vecs, vecs, sizeof(cplx) * (size_t)g->lv[l].nv * g->lv[l].n);
    return build_level(g, l, (const cplx *)vecs, g->lv[l].nv);
}

/* the null vectors of level l as the setup left them (normalised, before
 * the chirality split and block orthonormalisation) */
void orc_mg_get_null_vectors(orc_mg *g, int l, double *out)
{
    memcpy(out, g->lv[l].vecs, sizeof(cplx) * (size_t)g->lv[l].nv * g->lv[l].n);
}

/* exact coarse mass shift: D_hat(m) = D_hat(m0) + (m - m0) 1, since
 * P^dag P = 1 and D(m) = D(0) + m */
void orc_mg_set_mass(orc_mg *g, double m)
{
    double dm = m - g->m;
    g->lv[0].op.m = m;
    for (int l = 1; l < g->nl; l++) {
        orc_lvl *C = &g->lv[l];
        int n = C->op.dof;
        for (long s = 0; s < C->op.nsite; s++)
            for (int r = 0; r < n; r++) C->Ybuf[((size_t)s * 9) * n * n + r * n + r] += dm;
    }
    g->m = m;
}

long orc_mg_solve(orc_mg *g, const double *b, double *x, double tol, orc_stats *st)
{
    orc_stats loc;
    memset(&loc, 0, sizeof(loc));
    vzero(g->lv[0].n, (cplx *)x);
    long it = gcr(g, 0, (const cplx *)b, (cplx *)x, tol, g->p.maxiter, pc_cycle, &loc);
    if (st) *st = loc;
    return it;
}

/* red/black solve: flexible GCR on S x_e = b_e - D_eo D_oo^-1 b_o with the
 * preconditioner [M (r_e, 0)]_e, stopped when |r_e| <= tol |b| (r_e is the
 * whole residual of D x = b once x_o = D_oo^-1 (b_o - D_oe x_e)); then x_o. */
long orc_mg_solve_eo(orc_mg *g, const double *bd, double *xd, double tol, orc_stats *st)
{
    const orc_op *A = &g->lv[0].op;
    long V = A->nsite, n = V * 12;
    double m = A->m;
    const cplx *b = (const cplx *)bd;
    cplx *x = (cplx *)xd;
    cplx *bo = valloc(n), *t = valloc(n), *be = valloc(n);
    orc_stats loc;
    memset(&loc, 0, sizeof(loc));
    for (long s = 0; s < V; s++)
        if (orc_parity(A->L, s)) memcpy(bo + 12 * s, b + 12 * s, sizeof(cplx) * 12);
    orc_wilson_hop_parity(A->L, (const double *)g->U, m, (const double *)bo, (double *)t, 0); /* D_eo b_o */
    for (long s = 0; s < V; s++)
        for (int c = 0; c < 12; c++)
            be[12 * s + c] = orc_parity(A->L, s) ? 0 : b[12 * s + c] - t[12 * s + c] / (4.0 + m);
    vzero(n, x);
    long it = gcr_op(g, 0, be, x, tol, g->p.maxiter, pc_cycle_even, schur_apply_lvl, sqrt(vnorm2(n, b)), &loc);
    /* x_o = (b_o - D_oe x_e) / (4+m) */
    orc_wilson_hop_parity(A->L, (const double *)g->U, m, (const double *)x, (double *)t, 1);
    for (long s = 0; s < V; s++)
        if (orc_parity(A->L, s))
            for (int c = 0; c < 12; c++) x[12 * s + c] = (b[12 * s + c] - t[12 * s + c]) / (4.0 + m);
    /* true residual of D x = b */
    op_apply(A, x, t);
    for (long i = 0; i < n; i++) t[i] = b[i] - t[i];
    double bn = sqrt(vnorm2(n, b));
    loc.true_relres = bn > 0 ? sqrt(vnorm2(n, t)) / bn : 0;
    loc.converged = loc.true_relres <= tol;
    if (st) *st = loc;
    free(bo); free(t); free(be);
    return it;
}

/* single preconditioner application z = M r (for parity of one cycle) */
void orc_mg_cycle(orc_mg *g, const double *r, double *z)
{
    mg_cycle(g, 0, (const cplx *)r, (cplx *)z, NULL);
}

int orc_mg_level_info(orc_mg *g, int l, int *L, int *dof, int *nv)
{
    if (l < 0 || l >= g->nl) return -1;
    memcpy(L, g->lv[l].op.L, sizeof(int) * 4);
    *dof = g->lv[l].op.dof;
    *nv = l + 1 < g->nl ? g->lv[l].nv : 0;
    return 0;
}

void orc_mg_get_P(orc_mg *g, int l, double *out)
{
    memcpy(out, g->lv[l].P, sizeof(cplx) * (size_t)g->lv[l].nv * g->lv[l].n);
}

void orc_mg_get_Y(orc_mg *g, int l, double *out)
{
    orc_lvl *C = &g->lv[l];
    memcpy(out, C->Ybuf, sizeof(cplx) * (size_t)C->op.nsite * 9 * C->op.dof * C->op.dof);
}

/* ---------------------------------------------------------------------- */
/* standalone solvers on the Wilson operator                                */
/* ---------------------------------------------------------------------- */
/* plain BiCGStab (van der Vorst 1992) on D x = b, x0 = 0: the unigrid
 * Krylov baseline; returns iterations (each costs two D applies). */
long orc_bicgstab(const int L[4], const double *U, double m, const double *bd, double *xd, double tol,
                  int maxiter, double *relres)
{
    orc_op A = {{L[0], L[1], L[2], L[3]}, vol(L), 12, 0, (const cplx *)U, m, NULL};
    long n = A.nsite * 12;
    const cplx *b = (const cplx *)bd;
    cplx *x = (cplx *)xd;
    cplx *r = valloc(n), *rh = valloc(n), *p = valloc(n), *v = valloc(n), *s = valloc(n), *t = valloc(n);
    vzero(n, x);
    vcopy(n, b, r);
    vcopy(n, b, rh);
    double bn = sqrt(vnorm2(n, b));
    cplx rho = 1, al = 1, om = 1;
    long it = 0;
    double rn = bn;
    while (rn > tol * bn && it < maxiter) {
        cplx rho1 = vdot(n, rh, r);
        if (rho1 == 0) break;
        cplx be = (rho1 / rho) * (al / om);
        for (long i = 0; i < n; i++) p[i] = r[i] + be * (p[i] - om * v[i]);
        op_apply(&A, p, v);
        al = rho1 / vdot(n, rh, v);
        for (long i = 0; i < n; i++) s[i] = r[i] - al * v[i];
        op_apply(&A, s, t);
        double tt = vnorm2(n, t);
        om = tt > 0 ? vdot(n, t, s) / tt : 0;
        for (long i = 0; i < n; i++) {
            x[i] += al * p[i] + om * s[i];
            r[i] = s[i] - om * t[i];
        }
        rho = rho1;
        it++;
        rn = sqrt(vnorm2(n, r));
        if (om == 0) break;
    }
    op_apply(&A, x, t);
    for (long i = 0; i < n; i++) t[i] = b[i] - t[i];
    if (relres) *relres = sqrt(vnorm2(n, t)) / bn;
    free(r); free(rh); free(p); free(v); free(s); free(t);
    return it;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* thread count of the following parallel regions (timing of the oracle) */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* standalone CGNR on a coarse stencil (for the oracle's own pins) */
long orc_cgnr_coarse(const int L[4], int dof, const double *Y, const double *b, double *x, double tol, int maxiter)
{
    orc_op A = {{L[0], L[1], L[2], L[3]}, vol(L), dof, 1, NULL, 0, (const cplx *)Y};
    return cgnr(&A, (const cplx *)b, (cplx *)x, tol, maxiter);
}

/* standalone MR smoothing on the Wilson operator; res[k] = |r - D e| after
 * k steps (k = 0..nsteps) */
void orc_mr_wilson(const int L[4], const double *U, double m, const double *r, double *e, int nsteps, double *res)
{
    orc_mg g;
    memset(&g, 0, sizeof(g));
    g.nl = 1;
    memcpy(g.lv[0].op.L, L, sizeof(int) * 4);
    g.lv[0].op.nsite = vol(L);
    g.lv[0].op.dof = 12;
    g.lv[0].op.kind = 0;
    g.lv[0].op.U = (const cplx *)U;
    g.lv[0].op.m = m;
    g.lv[0].n = vol(L) * 12;
    long n = g.lv[0].n;
    cplx *t = valloc(n);
    for (int k = 0; k <= nsteps; k++) {
        if (k > 0) mr_smooth(&g, 0, (const cplx *)r, (cplx *)e, 1, NULL);
        op_apply(&g.lv[0].op, (const cplx *)e, t);
        for (long i = 0; i < n; i++) t[i] = ((const cplx *)r)[i] - t[i];
        res[k] = sqrt(vnorm2(n, t));
    }
    free(t);
}
