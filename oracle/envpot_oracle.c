/*
 * FP64 CPU oracle for the environment electrostatic potential.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
 * the CPU-baseline leg of the benchmark may load this file.  It shares no
 * code with the HIP library: its own Boys function, normalisation, overlap,
 * Hermite expansion and summation, written as plainly as the definitions.
 *
 * What it computes (paper Sec. II.B, Eq. ElectrostaticField, with the
 * electron density given by a density matrix over Gaussian basis functions
 * instead of the paper's point-charge cells):
 *
 *     V(r)  = V_nuc(r) - V_ele(r)
 *     V_nuc = sum_A Z_A / |r - R_A|
 *     V_ele = sum_{mu,nu} P_{mu nu} [mu nu | r],
 *     [mu nu | r] = integral chi_mu(r') chi_nu(r') / |r' - r| d^3 r'
 *
 * The paper's U_ES of Eq. ElectrostaticField is -V (it is the potential energy
 * of an electron; V is the electrostatic potential).
 *
 * oracle_field gives the field E = -grad V of the same environment (an
 * extension: the paper uses only the potential), from the derivative of the
 * Hermite integrals with respect to the point, R_{t+1,u,v} etc.
 *
 * Every [mu nu | r] is evaluated per Cartesian component pair and per
 * primitive pair by the McMurchie-Davidson scheme (textbook: McMurchie and
 * Davidson 1978; Helgaker, Joergensen, Olsen 2000, Sec. 9.5 and 9.9):
 *   [a b | C] = (2 pi / p) sum_{tuv} E^{ij}_t E^{kl}_u E^{mn}_v R_{tuv}(p, P - C)
 * with no folding of the density matrix into the Hermite coefficients.
 *
 * Boys function: power series below T = 30, erf plus upward recursion above
 * (a method that differs on purpose from the tabulated one of the library).
 * Overlaps: binomial expansion about the product centre (again different from
 * the E-recursion used for the potential).
 *
 * Sums are Neumaier-compensated; V_nuc and V_ele are summed separately and
 * the conditioning scale A(r) = V_nuc + sum |terms| is returned with them.
 *
 * Parity against numbers printed in the paper is unpinned: the paper prints
 * no potential values.  The pins are closed forms, invariants and brute-force
 * quadrature (tests/test_oracle_*.py).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_LMAX 2           /* s, p, d shells */
#define ORACLE_LSUM (2 * ORACLE_LMAX)
#define ORACLE_NMAXCART 6

static const double PI = 3.14159265358979323846;

/* Deliberate mistakes for the mutation tests (0 = none).  A mutation is a
 * wrong variant of one formula; the tests check that some pin catches it. */
static int g_mutation = 0;
void oracle_set_mutation(int m) { g_mutation = m; }
int oracle_get_mutation(void) { return g_mutation; }

/* ---------------------------------------------------------------- helpers */

static double dfact(int n) { /* double factorial, (-1)!! = 0!! = 1 */
    double r = 1.0;
    for (int k = n; k > 1; k -= 2) r *= (double)k;
    return r;
}

static double binom(int n, int k) {
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (double)(n - k + i) / (double)i;
    return r;
}

typedef struct { double s, c; } nsum; /* Neumaier running sum */

static void nsum_add(nsum* a, double x) {
    double t = a->s + x;
    if (!isfinite(t)) { a->s = t; return; } /* a point on a nucleus: +inf */
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static double nsum_get(const nsum* a) { return isfinite(a->s) ? a->s + a->c : a->s; }

/* Cartesian exponents of component c of a shell of angular momentum l,
 * x-major lexicographic: p = x,y,z; d = xx,xy,xz,yy,yz,zz. */
static void cart_exps(int l, int c, int e[3]) {
    int idx = 0;
    for (int i = l; i >= 0; --i)
        for (int j = l - i; j >= 0; --j) {
            if (idx == c) { e[0] = i; e[1] = j; e[2] = l - i - j; return; }
            ++idx;
        }
    e[0] = e[1] = e[2] = -1;
}

static int ncart(int l) { return (l + 1) * (l + 2) / 2; }

/* --------------------------------------------------------- Boys function */

/* F_n(T) = integral_0^1 t^{2n} exp(-T t^2) dt.
 * T <= 30: F_n = exp(-T) sum_{i>=0} (2T)^i / ((2n+1)(2n+3)...(2n+2i+1)),
 *          summed until a term falls below 1e-17 of the sum.
 * T  > 30: F_0 = (sqrt(pi)/2) erf(sqrt T)/sqrt T, then upward
 *          F_{n+1} = ((2n+1) F_n - exp(-T)) / (2T). */
void oracle_boys(int nmax, double T, double* F) {
    if (T <= 30.0) {
        double e = exp(-T);
        for (int n = 0; n <= nmax; ++n) {
            double term = 1.0 / (2.0 * n + 1.0);
            double sum = term;
            for (int i = 1; i < 1000; ++i) {
                term *= 2.0 * T / (2.0 * n + 2.0 * i + 1.0);
                sum += term;
                if (term < 1e-17 * sum) break;
            }
            F[n] = e * sum;
        }
    } else {
        double st = sqrt(T), e = exp(-T);
        F[0] = 0.5 * sqrt(PI) * erf(st) / st;
        if (g_mutation == 5) F[0] = 0.5 * sqrt(PI) / st / st;
        for (int n = 0; n < nmax; ++n)
            F[n + 1] = ((2.0 * n + 1.0) * F[n] - e) / (2.0 * T);
    }
}

/* ---------------------------------------------------------- normalisation */

/* Primitive Cartesian Gaussian normalisation
 * N = (2a/pi)^{3/4} (4a)^{(i+j+k)/2} / sqrt((2i-1)!! (2j-1)!! (2k-1)!!). */
double oracle_prim_norm(double a, int i, int j, int k) {
    double n = pow(2.0 * a / PI, 0.75) * pow(4.0 * a, 0.5 * (i + j + k)) /
               sqrt(dfact(2 * i - 1) * dfact(2 * j - 1) * dfact(2 * k - 1));
    if (g_mutation == 6) n = pow(2.0 * a / PI, 0.75);
    return n;
}

/* integral x^m exp(-p x^2) dx over R: 0 for odd m, (m-1)!!/(2p)^{m/2} sqrt(pi/p). */
static double moment1d(int m, double p) {
    if (m & 1) return 0.0;
    return dfact(m - 1) / pow(2.0 * p, 0.5 * m) * sqrt(PI / p);
}

/* Scale that makes the contracted component (i,j,k) of a shell have unit
 * self-overlap: 1/sqrt(sum_ab c_a c_b N_a N_b prod_d moment1d(2 e_d, a_a+a_b)). */
static double contracted_scale(int nprim, const double* ex, const double* co,
                               const int e[3]) {
    double s = 0.0;
    for (int a = 0; a < nprim; ++a)
        for (int b = 0; b < nprim; ++b) {
            double p = ex[a] + ex[b];
            s += co[a] * co[b] * oracle_prim_norm(ex[a], e[0], e[1], e[2]) *
                 oracle_prim_norm(ex[b], e[0], e[1], e[2]) * moment1d(2 * e[0], p) *
                 moment1d(2 * e[1], p) * moment1d(2 * e[2], p);
        }
    return 1.0 / sqrt(s);
}

/* ------------------------------------------------ overlap (binomial form) */

/* 1-D overlap integral (x-A)^i (x-B)^j exp(-a(x-A)^2 - b(x-B)^2) over R,
 * by expanding both monomials about the product centre P. */
double oracle_overlap1d(int i, int j, double a, double b, double A, double B) {
    double p = a + b, mu = a * b / p, P = (a * A + b * B) / p;
    double XPA = P - A, XPB = P - B, s = 0.0;
    for (int k = 0; k <= i; ++k)
        for (int l = 0; l <= j; ++l)
            s += binom(i, k) * binom(j, l) * pow(XPA, i - k) * pow(XPB, j - l) *
                 moment1d(k + l, p);
    return exp(-mu * (A - B) * (A - B)) * s;
}

/* ------------------------------------------------ Hermite E-coefficients */

/* E^{ij}_t for i <= imax, j <= jmax, t <= i+j of one Cartesian direction.
 * Layout E[(i*(jmax+1) + j)*(imax+jmax+1) + t]. */
static void hermite_E(int imax, int jmax, double a, double b, double A, double B,
                      double* E) {
    double p = a + b, mu = a * b / p, P = (a * A + b * B) / p;
    double XPA = P - A, XPB = P - B, XAB = A - B;
    int tw = imax + jmax + 1;
#define EI(i, j, t) E[((i) * (jmax + 1) + (j)) * tw + (t)]
    for (int k = 0; k < (imax + 1) * (jmax + 1) * tw; ++k) E[k] = 0.0;
    if (g_mutation == 2) XPA = -XPA;
    if (g_mutation == 3) XPA = XPB;
    EI(0, 0, 0) = exp(-mu * XAB * XAB);
    for (int i = 0; i <= imax; ++i)
        for (int j = 0; j <= jmax; ++j) {
            if (i == 0 && j == 0) continue;
            for (int t = 0; t <= i + j; ++t) {
                double v;
                if (i > 0) { /* raise i from (i-1, j) */
                    double em = (t > 0) ? EI(i - 1, j, t - 1) : 0.0;
                    double e0 = (t <= i - 1 + j) ? EI(i - 1, j, t) : 0.0;
                    double ep = (t + 1 <= i - 1 + j) ? EI(i - 1, j, t + 1) : 0.0;
                    if (g_mutation == 1) ep = 0.0;
                    v = em / (2.0 * p) + XPA * e0 + (t + 1) * ep;
                } else {     /* raise j from (i, j-1) */
                    double em = (t > 0) ? EI(i, j - 1, t - 1) : 0.0;
                    double e0 = (t <= i + j - 1) ? EI(i, j - 1, t) : 0.0;
                    double ep = (t + 1 <= i + j - 1) ? EI(i, j - 1, t + 1) : 0.0;
                    if (g_mutation == 1) ep = 0.0;
                    v = em / (2.0 * p) + XPB * e0 + (t + 1) * ep;
                }
                EI(i, j, t) = v;
            }
        }
#undef EI
}

/* Single coefficient, for tests. */
double oracle_hermite_E(int i, int j, int t, double a, double b, double A, double B) {
    double E[(ORACLE_LMAX + 3) * (ORACLE_LMAX + 3) * (2 * ORACLE_LMAX + 5)];
    if (i < 0 || j < 0 || i > ORACLE_LMAX + 2 || j > ORACLE_LMAX + 2) return NAN;
    if (t < 0 || t > i + j) return 0.0;
    hermite_E(i, j, a, b, A, B, E);
    return E[(i * (j + 1) + j) * (i + j + 1) + t];
}

/* --------------------------------------------- Hermite Coulomb integrals */

#define RDIM (ORACLE_LSUM + 2)  /* one order more than V needs: the field */
#define RIDX(n, t, u, v) ((((n) * RDIM + (t)) * RDIM + (u)) * RDIM + (v))

/* R^n_{tuv}(p, X, Y, Z) for n+t+u+v <= L; returns R^0_{tuv} in out[t][u][v]
 * (layout (t*RDIM+u)*RDIM+v).  X = P_x - C_x etc.
 *   R^n_000 = (-2p)^n F_n(p (X^2+Y^2+Z^2))
 *   R^n_{t+1,u,v} = t R^{n+1}_{t-1,u,v} + X R^{n+1}_{t,u,v}  (same for u, v) */
void oracle_hermite_R(int L, double p, double X, double Y, double Z, double* out) {
    double R[RDIM * RDIM * RDIM * RDIM];
    double F[RDIM + 1];
    oracle_boys(L, p * (X * X + Y * Y + Z * Z), F);
    for (int n = L; n >= 0; --n) {
        for (int t = 0; t <= L - n; ++t)
            for (int u = 0; u <= L - n - t; ++u)
                for (int v = 0; v <= L - n - t - u; ++v) {
                    double r;
                    if (t > 0) {
                        r = X * R[RIDX(n + 1, t - 1, u, v)];
                        if (t > 1) r += (t - 1) * R[RIDX(n + 1, t - 2, u, v)];
                    } else if (u > 0) {
                        r = Y * R[RIDX(n + 1, t, u - 1, v)];
                        if (u > 1) r += (u - 1) * R[RIDX(n + 1, t, u - 2, v)];
                    } else if (v > 0) {
                        r = Z * R[RIDX(n + 1, t, u, v - 1)];
                        if (v > 1) r += (v - 1) * R[RIDX(n + 1, t, u, v - 2)];
                    } else {
                        r = pow(-2.0 * p, n) * F[n];
                    }
                    if (g_mutation == 4 && (t + u + v) == 1) r = -r;
                    R[RIDX(n, t, u, v)] = r;
                }
    }
    for (int t = 0; t <= L; ++t)
        for (int u = 0; u <= L - t; ++u)
            for (int v = 0; v <= L - t - u; ++v)
                out[(t * RDIM + u) * RDIM + v] = R[RIDX(0, t, u, v)];
}

/* ------------------------------------------------------------ the input */

typedef struct {
    int K;                 /* nuclei */
    const double* xyz;     /* K x 3 */
    const double* Z;       /* K */
    int S;                 /* shells */
    const int32_t* atom;   /* S: centre = xyz[atom] */
    const int32_t* l;      /* S */
    const int32_t* nprim;  /* S */
    const int64_t* poff;   /* S: offset into ex / co */
    const double* ex;
    const double* co;
    int nbf;
    const int64_t* rowp;   /* CSR P: nbf+1 */
    const int32_t* col;
    const double* val;
} oracle_env;

/* One ordered shell pair with a nonzero density block. */
typedef struct {
    int I, J;
    double* Pblk;          /* ncart(lI) x ncart(lJ), scaled by component norms */
} shellpair;

typedef struct {
    int n;
    shellpair* sp;
    int* bf0;              /* first basis function of each shell */
    double** cscale;       /* per shell: contracted component scales */
} prepared;

static int shell_of_bf(const int* bf0, int S, int mu) {
    int lo = 0, hi = S - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) / 2;
        if (bf0[mid] <= mu) lo = mid; else hi = mid - 1;
    }
    return lo;
}

static void prepare(const oracle_env* e, prepared* pr) {
    pr->bf0 = (int*)malloc(sizeof(int) * (e->S + 1));
    pr->cscale = (double**)malloc(sizeof(double*) * (e->S > 0 ? e->S : 1));
    int b = 0;
    for (int s = 0; s < e->S; ++s) {
        pr->bf0[s] = b;
        int nc = ncart(e->l[s]);
        pr->cscale[s] = (double*)malloc(sizeof(double) * nc);
        for (int c = 0; c < nc; ++c) {
            int ce[3];
            cart_exps(e->l[s], c, ce);
            pr->cscale[s][c] = contracted_scale(e->nprim[s], e->ex + e->poff[s],
                                                e->co + e->poff[s], ce);
        }
        b += nc;
    }
    pr->bf0[e->S] = b;
    /* dense blocks of every ordered shell pair that has a nonzero element */
    int cap = 64;
    pr->sp = (shellpair*)malloc(sizeof(shellpair) * cap);
    pr->n = 0;
    int* last = (int*)malloc(sizeof(int) * (e->S > 0 ? e->S : 1));
    int* slot = (int*)malloc(sizeof(int) * (e->S > 0 ? e->S : 1));
    for (int s = 0; s < e->S; ++s) last[s] = -1;
    for (int I = 0; I < e->S; ++I) {
        int nI = ncart(e->l[I]);
        for (int ci = 0; ci < nI; ++ci) {
            int mu = pr->bf0[I] + ci;
            for (int64_t k = e->rowp[mu]; k < e->rowp[mu + 1]; ++k) {
                int nu = e->col[k];
                double v = e->val[k];
                if (v == 0.0) continue;
                int J = shell_of_bf(pr->bf0, e->S, nu);
                if (last[J] != I) {
                    if (pr->n == cap) {
                        cap *= 2;
                        pr->sp = (shellpair*)realloc(pr->sp, sizeof(shellpair) * cap);
                    }
                    last[J] = I;
                    slot[J] = pr->n;
                    shellpair* q = &pr->sp[pr->n++];
                    q->I = I; q->J = J;
                    q->Pblk = (double*)calloc((size_t)nI * ncart(e->l[J]), sizeof(double));
                }
                shellpair* q = &pr->sp[slot[J]];
                int cj = nu - pr->bf0[J];
                q->Pblk[ci * ncart(e->l[J]) + cj] +=
                    v * pr->cscale[I][ci] * pr->cscale[J][cj];
            }
        }
    }
    free(last);
    free(slot);
}

static void release(const oracle_env* e, prepared* pr) {
    for (int k = 0; k < pr->n; ++k) free(pr->sp[k].Pblk);
    free(pr->sp);
    for (int s = 0; s < e->S; ++s) free(pr->cscale[s]);
    free(pr->cscale);
    free(pr->bf0);
}

/* Screening rule for primitive pair (a in I, b in J): dropped when
 * |c_a c_b| N0_a N0_b (pi/p)^{3/2} exp(-mu |A-B|^2) < thr,
 * N0 = (2 alpha/pi)^{3/4} (s-type primitive normalisation); P is not used. */
static int screened_out(double ca, double cb, double a, double b, double RAB2,
                        double thr) {
    double p = a + b, mu = a * b / p;
    double bound = fabs(ca * cb) * pow(2.0 * a / PI, 0.75) * pow(2.0 * b / PI, 0.75) *
                   pow(PI / p, 1.5) * exp(-mu * RAB2);
    return bound < thr;
}

/* Potential at one point. */
static void potential_one(const oracle_env* e, const prepared* pr, const double* r,
                          int screen, double thr, double out[4]) {
    nsum vn = {0, 0}, ve = {0, 0};
    double absterms = 0.0;
    for (int A = 0; A < e->K; ++A) {
        double dx = r[0] - e->xyz[3 * A], dy = r[1] - e->xyz[3 * A + 1],
               dz = r[2] - e->xyz[3 * A + 2];
        nsum_add(&vn, e->Z[A] / sqrt(dx * dx + dy * dy + dz * dz));
    }
    double Ex[(ORACLE_LMAX + 1) * (ORACLE_LMAX + 1) * (ORACLE_LSUM + 1)];
    double Ey[(ORACLE_LMAX + 1) * (ORACLE_LMAX + 1) * (ORACLE_LSUM + 1)];
    double Ez[(ORACLE_LMAX + 1) * (ORACLE_LMAX + 1) * (ORACLE_LSUM + 1)];
    double R[RDIM * RDIM * RDIM];
    for (int k = 0; k < pr->n; ++k) {
        const shellpair* q = &pr->sp[k];
        int I = q->I, J = q->J, lI = e->l[I], lJ = e->l[J];
        const double* A = e->xyz + 3 * e->atom[I];
        const double* B = e->xyz + 3 * e->atom[J];
        double RAB2 = (A[0] - B[0]) * (A[0] - B[0]) + (A[1] - B[1]) * (A[1] - B[1]) +
                      (A[2] - B[2]) * (A[2] - B[2]);
        int nI = ncart(lI), nJ = ncart(lJ), tw = lI + lJ + 1;
        for (int pa = 0; pa < e->nprim[I]; ++pa)
            for (int pb = 0; pb < e->nprim[J]; ++pb) {
                double a = e->ex[e->poff[I] + pa], b = e->ex[e->poff[J] + pb];
                double ca = e->co[e->poff[I] + pa], cb = e->co[e->poff[J] + pb];
                if (screen && screened_out(ca, cb, a, b, RAB2, thr)) continue;
                double p = a + b;
                double P[3] = {(a * A[0] + b * B[0]) / p, (a * A[1] + b * B[1]) / p,
                               (a * A[2] + b * B[2]) / p};
                hermite_E(lI, lJ, a, b, A[0], B[0], Ex);
                hermite_E(lI, lJ, a, b, A[1], B[1], Ey);
                hermite_E(lI, lJ, a, b, A[2], B[2], Ez);
                oracle_hermite_R(lI + lJ, p, P[0] - r[0], P[1] - r[1], P[2] - r[2], R);
                double pref = 2.0 * PI / p;
                for (int ci = 0; ci < nI; ++ci) {
                    int ei[3];
                    cart_exps(lI, ci, ei);
                    double Na = oracle_prim_norm(a, ei[0], ei[1], ei[2]);
                    for (int cj = 0; cj < nJ; ++cj) {
                        double Pmn = q->Pblk[ci * nJ + cj];
                        if (Pmn == 0.0) continue;
                        int ej[3];
                        cart_exps(lJ, cj, ej);
                        double Nb = oracle_prim_norm(b, ej[0], ej[1], ej[2]);
                        double s = 0.0;
                        for (int t = 0; t <= ei[0] + ej[0]; ++t)
                            for (int u = 0; u <= ei[1] + ej[1]; ++u)
                                for (int v = 0; v <= ei[2] + ej[2]; ++v)
                                    s += Ex[(ei[0] * (lJ + 1) + ej[0]) * tw + t] *
                                         Ey[(ei[1] * (lJ + 1) + ej[1]) * tw + u] *
                                         Ez[(ei[2] * (lJ + 1) + ej[2]) * tw + v] *
                                         R[(t * RDIM + u) * RDIM + v];
                        double term = Pmn * ca * cb * Na * Nb * pref * s;
                        nsum_add(&ve, term);
                        absterms += fabs(term);
                    }
                }
            }
    }
    double vnuc = nsum_get(&vn), vele = nsum_get(&ve);
    out[0] = vnuc - vele;
    out[1] = vnuc;
    out[2] = vele;
    out[3] = vnuc + absterms;
}

/* Potential at n points.  out is n x 4: V, V_nuc, V_ele, A.
 * screen != 0 applies the primitive-pair screening rule with threshold thr.
 * nthreads > 0 caps the OpenMP team (0: library default).
 * Returns 0, or -1 on a bad argument (l outside 0..2). */
int oracle_potential(int K, const double* xyz, const double* Z, int S,
                     const int32_t* atom, const int32_t* l, const int32_t* nprim,
                     const int64_t* poff, const double* ex, const double* co, int nbf,
                     const int64_t* rowp, const int32_t* col, const double* val,
                     int64_t n, const double* pts, int screen, double thr,
                     int nthreads, double* out) {
    for (int s = 0; s < S; ++s)
        if (l[s] < 0 || l[s] > ORACLE_LMAX) return -1;
    oracle_env e = {K, xyz, Z, S, atom, l, nprim, poff, ex, co, nbf, rowp, col, val};
    prepared pr;
    prepare(&e, &pr);
#ifdef _OPENMP
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
#else
    (void)nthreads;
#endif
    for (int64_t i = 0; i < n; ++i) potential_one(&e, &pr, pts + 3 * i, screen, thr, out + 4 * i);
    release(&e, &pr);
    return 0;
}

/* Field at one point, E = -grad V (same input and pair loop as
 * potential_one).  With X = P - r, the Hermite integrals R_tuv are
 * derivatives with respect to P, and moving r moves X the other way:
 *   d/dr_x [a b | r] = -(2 pi / p) sum_tuv E_t E_u E_v R_{t+1,u,v}(p, X),
 * likewise y (u+1) and z (v+1).  Hence
 *   E(r) = sum_A Z_A (r - R_A) / |r - R_A|^3
 *          - sum_{mu nu} P_{mu nu} (2 pi / p) sum_tuv E E E (R_{t+1,u,v}, R_{t,u+1,v}, R_{t,u,v+1}),
 * which needs R up to total order l_I + l_J + 1.
 * out[0..2] = E, out[3] = AE = sum_A Z_A / |r - R_A|^2 + sum over terms of
 * the Euclidean length of each term's vector (the conditioning scale). */
static void field_one(const oracle_env* e, const prepared* pr, const double* r,
                      int screen, double thr, double out[4]) {
    nsum ex = {0, 0}, ey = {0, 0}, ez = {0, 0};
    double absterms = 0.0;
    for (int A = 0; A < e->K; ++A) {
        double dx = r[0] - e->xyz[3 * A], dy = r[1] - e->xyz[3 * A + 1],
               dz = r[2] - e->xyz[3 * A + 2];
        double d2 = dx * dx + dy * dy + dz * dz, d = sqrt(d2);
        double f = e->Z[A] / (d2 * d);
        nsum_add(&ex, f * dx);
        nsum_add(&ey, f * dy);
        nsum_add(&ez, f * dz);
        absterms += fabs(e->Z[A]) / d2;
    }
    double Ex[(ORACLE_LMAX + 1) * (ORACLE_LMAX + 1) * (ORACLE_LSUM + 1)];
    double Ey[(ORACLE_LMAX + 1) * (ORACLE_LMAX + 1) * (ORACLE_LSUM + 1)];
    double Ez[(ORACLE_LMAX + 1) * (ORACLE_LMAX + 1) * (ORACLE_LSUM + 1)];
    double R[RDIM * RDIM * RDIM];
    for (int k = 0; k < pr->n; ++k) {
        const shellpair* q = &pr->sp[k];
        int I = q->I, J = q->J, lI = e->l[I], lJ = e->l[J];
        const double* A = e->xyz + 3 * e->atom[I];
        const double* B = e->xyz + 3 * e->atom[J];
        double RAB2 = (A[0] - B[0]) * (A[0] - B[0]) + (A[1] - B[1]) * (A[1] - B[1]) +
                      (A[2] - B[2]) * (A[2] - B[2]);
        int nI = ncart(lI), nJ = ncart(lJ), tw = lI + lJ + 1;
        for (int pa = 0; pa < e->nprim[I]; ++pa)
            for (int pb = 0; pb < e->nprim[J]; ++pb) {
                double a = e->ex[e->poff[I] + pa], b = e->ex[e->poff[J] + pb];
                double ca = e->co[e->poff[I] + pa], cb = e->co[e->poff[J] + pb];
                if (screen && screened_out(ca, cb, a, b, RAB2, thr)) continue;
                double p = a + b;
                double P[3] = {(a * A[0] + b * B[0]) / p, (a * A[1] + b * B[1]) / p,
                               (a * A[2] + b * B[2]) / p};
                hermite_E(lI, lJ, a, b, A[0], B[0], Ex);
                hermite_E(lI, lJ, a, b, A[1], B[1], Ey);
                hermite_E(lI, lJ, a, b, A[2], B[2], Ez);
                oracle_hermite_R(lI + lJ + 1, p, P[0] - r[0], P[1] - r[1], P[2] - r[2], R);
                double pref = 2.0 * PI / p;
                for (int ci = 0; ci < nI; ++ci) {
                    int ei[3];
                    cart_exps(lI, ci, ei);
                    double Na = oracle_prim_norm(a, ei[0], ei[1], ei[2]);
                    for (int cj = 0; cj < nJ; ++cj) {
                        double Pmn = q->Pblk[ci * nJ + cj];
                        if (Pmn == 0.0) continue;
                        int ej[3];
                        cart_exps(lJ, cj, ej);
                        double Nb = oracle_prim_norm(b, ej[0], ej[1], ej[2]);
                        double gx = 0.0, gy = 0.0, gz = 0.0;
                        for (int t = 0; t <= ei[0] + ej[0]; ++t)
                            for (int u = 0; u <= ei[1] + ej[1]; ++u)
                                for (int v = 0; v <= ei[2] + ej[2]; ++v) {
                                    double E3 = Ex[(ei[0] * (lJ + 1) + ej[0]) * tw + t] *
                                                Ey[(ei[1] * (lJ + 1) + ej[1]) * tw + u] *
                                                Ez[(ei[2] * (lJ + 1) + ej[2]) * tw + v];
                                    if (g_mutation == 7) gx += E3 * R[(t * RDIM + u + 1) * RDIM + v];
                                    else gx += E3 * R[((t + 1) * RDIM + u) * RDIM + v];
                                    gy += E3 * R[(t * RDIM + u + 1) * RDIM + v];
                                    gz += E3 * R[(t * RDIM + u) * RDIM + v + 1];
                                }
                        double c = Pmn * ca * cb * Na * Nb * pref;
                        if (g_mutation == 8) c = -c;
                        nsum_add(&ex, -c * gx);
                        nsum_add(&ey, -c * gy);
                        nsum_add(&ez, -c * gz);
                        absterms += fabs(c) * sqrt(gx * gx + gy * gy + gz * gz);
                    }
                }
            }
    }
    out[0] = nsum_get(&ex);
    out[1] = nsum_get(&ey);
    out[2] = nsum_get(&ez);
    out[3] = absterms;
}

/* Field E = -grad V at n points.  out is n x 4: E_x, E_y, E_z, AE.
 * Arguments and return value as oracle_potential. */
int oracle_field(int K, const double* xyz, const double* Z, int S,
                 const int32_t* atom, const int32_t* l, const int32_t* nprim,
                 const int64_t* poff, const double* ex, const double* co, int nbf,
                 const int64_t* rowp, const int32_t* col, const double* val,
                 int64_t n, const double* pts, int screen, double thr,
                 int nthreads, double* out) {
    for (int s = 0; s < S; ++s)
        if (l[s] < 0 || l[s] > ORACLE_LMAX) return -1;
    oracle_env e = {K, xyz, Z, S, atom, l, nprim, poff, ex, co, nbf, rowp, col, val};
    prepared pr;
    prepare(&e, &pr);
#ifdef _OPENMP
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
#else
    (void)nthreads;
#endif
    for (int64_t i = 0; i < n; ++i) field_one(&e, &pr, pts + 3 * i, screen, thr, out + 4 * i);
    release(&e, &pr);
    return 0;
}

/* Row contributions of tr(P S): out[mu] = sum_nu P_{mu nu} S_{mu nu}, with S
 * the overlap of the normalised contracted basis (binomial form). */
int oracle_density_overlap_rows(int K, const double* xyz, int S, const int32_t* atom,
                                const int32_t* l, const int32_t* nprim,
                                const int64_t* poff, const double* ex,
                                const double* co, int nbf, const int64_t* rowp,
                                const int32_t* col, const double* val, double* out) {
    for (int s = 0; s < S; ++s)
        if (l[s] < 0 || l[s] > ORACLE_LMAX) return -1;
    (void)K;
    oracle_env e = {K, xyz, NULL, S, atom, l, nprim, poff, ex, co, nbf, rowp, col, val};
    prepared pr;
    prepare(&e, &pr);
    for (int mu = 0; mu < nbf; ++mu) out[mu] = 0.0;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int k = 0; k < pr.n; ++k) {
        double Sx[(ORACLE_LMAX + 1) * (ORACLE_LMAX + 1)], Sy[(ORACLE_LMAX + 1) * (ORACLE_LMAX + 1)],
            Sz[(ORACLE_LMAX + 1) * (ORACLE_LMAX + 1)];
        const shellpair* q = &pr.sp[k];
        int I = q->I, J = q->J, nI = ncart(l[I]), nJ = ncart(l[J]);
        const double* A = xyz + 3 * atom[I];
        const double* B = xyz + 3 * atom[J];
        double* acc = (double*)calloc((size_t)nI * nJ, sizeof(double));
        int eI[ORACLE_NMAXCART][3], eJ[ORACLE_NMAXCART][3];
        for (int ci = 0; ci < nI; ++ci) cart_exps(l[I], ci, eI[ci]);
        for (int cj = 0; cj < nJ; ++cj) cart_exps(l[J], cj, eJ[cj]);
        for (int pa = 0; pa < nprim[I]; ++pa)
            for (int pb = 0; pb < nprim[J]; ++pb) {
                double a = ex[poff[I] + pa], b = ex[poff[J] + pb];
                double Na[ORACLE_NMAXCART], Nb[ORACLE_NMAXCART];
                for (int ci = 0; ci < nI; ++ci) Na[ci] = oracle_prim_norm(a, eI[ci][0], eI[ci][1], eI[ci][2]);
                for (int cj = 0; cj < nJ; ++cj) Nb[cj] = oracle_prim_norm(b, eJ[cj][0], eJ[cj][1], eJ[cj][2]);
                /* the 1-D overlaps of this primitive pair, for every exponent pair */
                for (int i = 0; i <= l[I]; ++i)
                    for (int j = 0; j <= l[J]; ++j) {
                        Sx[i * (ORACLE_LMAX + 1) + j] = oracle_overlap1d(i, j, a, b, A[0], B[0]);
                        Sy[i * (ORACLE_LMAX + 1) + j] = oracle_overlap1d(i, j, a, b, A[1], B[1]);
                        Sz[i * (ORACLE_LMAX + 1) + j] = oracle_overlap1d(i, j, a, b, A[2], B[2]);
                    }
                for (int ci = 0; ci < nI; ++ci)
                    for (int cj = 0; cj < nJ; ++cj) {
                        if (q->Pblk[ci * nJ + cj] == 0.0) continue;
                        const int* ei = eI[ci];
                        const int* ej = eJ[cj];
                        acc[ci * nJ + cj] += co[poff[I] + pa] * co[poff[J] + pb] * Na[ci] * Nb[cj] *
                                             Sx[ei[0] * (ORACLE_LMAX + 1) + ej[0]] *
                                             Sy[ei[1] * (ORACLE_LMAX + 1) + ej[1]] *
                                             Sz[ei[2] * (ORACLE_LMAX + 1) + ej[2]];
                    }
            }
        for (int ci = 0; ci < nI; ++ci)
            for (int cj = 0; cj < nJ; ++cj) {
                const double v = q->Pblk[ci * nJ + cj] * acc[ci * nJ + cj];  /* Pblk holds the scales */
#ifdef _OPENMP
#pragma omp atomic
#endif
                out[pr.bf0[I] + ci] += v;
            }
        free(acc);
    }
    release(&e, &pr);
    return 0;
}

/* Overlap matrix of the normalised contracted basis (dense nbf x nbf). */
int oracle_overlap_matrix(const double* xyz, int S, const int32_t* atom,
                          const int32_t* l, const int32_t* nprim, const int64_t* poff,
                          const double* ex, const double* co, int nbf, double* Smat) {
    for (int s = 0; s < S; ++s)
        if (l[s] < 0 || l[s] > ORACLE_LMAX) return -1;
    int* bf0 = (int*)malloc(sizeof(int) * (S + 1));
    int b = 0;
    for (int s = 0; s < S; ++s) { bf0[s] = b; b += ncart(l[s]); }
    bf0[S] = b;
    if (b != nbf) { free(bf0); return -1; }
    for (int I = 0; I < S; ++I)
        for (int J = 0; J < S; ++J) {
            const double* A = xyz + 3 * atom[I];
            const double* B = xyz + 3 * atom[J];
            for (int ci = 0; ci < ncart(l[I]); ++ci)
                for (int cj = 0; cj < ncart(l[J]); ++cj) {
                    int ei[3], ej[3];
                    cart_exps(l[I], ci, ei);
                    cart_exps(l[J], cj, ej);
                    double si = contracted_scale(nprim[I], ex + poff[I], co + poff[I], ei);
                    double sj = contracted_scale(nprim[J], ex + poff[J], co + poff[J], ej);
                    double s = 0.0;
                    for (int pa = 0; pa < nprim[I]; ++pa)
                        for (int pb = 0; pb < nprim[J]; ++pb) {
                            double a = ex[poff[I] + pa], bb = ex[poff[J] + pb];
                            s += co[poff[I] + pa] * co[poff[J] + pb] *
                                 oracle_prim_norm(a, ei[0], ei[1], ei[2]) *
                                 oracle_prim_norm(bb, ej[0], ej[1], ej[2]) *
                                 oracle_overlap1d(ei[0], ej[0], a, bb, A[0], B[0]) *
                                 oracle_overlap1d(ei[1], ej[1], a, bb, A[1], B[1]) *
                                 oracle_overlap1d(ei[2], ej[2], a, bb, A[2], B[2]);
                        }
                    Smat[(size_t)(bf0[I] + ci) * nbf + bf0[J] + cj] = si * sj * s;
                }
        }
    free(bf0);
    return 0;
}

/* Number of primitive shell pairs the screened oracle keeps (unique, I<=J,
 * a<=b when I==J), for reporting the pair count of a workload. */
int64_t oracle_count_pairs(const double* xyz, int S, const int32_t* atom,
                           const int32_t* l, const int32_t* nprim, const int64_t* poff,
                           const double* ex, const double* co, int nbf,
                           const int64_t* rowp, const int32_t* col, const double* val,
                           int screen, double thr) {
    oracle_env e = {0, xyz, NULL, S, atom, l, nprim, poff, ex, co, nbf, rowp, col, val};
    prepared pr;
    prepare(&e, &pr);
    int64_t cnt = 0;
    for (int k = 0; k < pr.n; ++k) {
        int I = pr.sp[k].I, J = pr.sp[k].J;
        if (I > J) continue;
        const double* A = xyz + 3 * atom[I];
        const double* B = xyz + 3 * atom[J];
        double RAB2 = (A[0] - B[0]) * (A[0] - B[0]) + (A[1] - B[1]) * (A[1] - B[1]) +
                      (A[2] - B[2]) * (A[2] - B[2]);
        for (int pa = 0; pa < nprim[I]; ++pa)
            for (int pb = (I == J ? pa : 0); pb < nprim[J]; ++pb) {
                double a = ex[poff[I] + pa], b = ex[poff[J] + pb];
                if (screen && screened_out(co[poff[I] + pa], co[poff[J] + pb], a, b,
                                           RAB2, thr))
                    continue;
                ++cnt;
            }
    }
    release(&e, &pr);
    return cnt;
}
