/*
 * tersoff_oracle.c -- plain FP64 CPU oracle for the Tersoff potential.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this file's library.  It shares no
 * code, header, table or helper with the GPU library; the two meet only on
 * the seeded inputs.
 *
 * What it computes (Hoehnerbach, Ismail, Bientinesi, "The Tersoff many-body
 * potential: sustainable performance through vectorization"):
 *   Eq. (1)  E = 1/2 sum_i sum_{j != i, r_ij < R+D} f_C(r_ij) [f_R(r_ij) + b_ij f_A(r_ij)]
 *   Eq. (2)  b_ij = (1 + beta^eta zeta_ij^eta)^(-1/(2 eta))
 *   Eq. (3)  zeta_ij = sum_{k != i,j, r_ik < R+D} f_C(r_ik) g(theta_ijk) exp((lambda3 (r_ij - r_ik))^m)
 * and the forces F = -dE/dx by the chain rule through r_ij, zeta_ij and the
 * r_ik and angles that zeta_ij depends on (see oracle_compute).
 *
 * Readings where the paper is silent (it omits "trivial definitions"):
 *  - the factor 1/2 in Eq. (1) (each unordered bond is visited twice);
 *  - k != j in Eq. (3);
 *  - f_C(r) = 1 (r < R-D), 1/2 - 1/2 sin(pi/2 (r-R)/D) (R-D <= r < R+D), 0
 *    (evaluated as sin^2(pi/4 (R+D-r)/D), see cutoff_fn);
 *    f_R = A exp(-lambda1 r); f_A = -B exp(-lambda2 r);
 *    g(theta) = gamma (1 + c^2/d^2 - c^2/(d^2 + (cos theta - h)^2));
 *  - the exponent of Eq. (3) is (lambda3 (r_ij - r_ik))^m, m in {1, 3}
 *    (m = 1 is the printed form);
 *  - multi-species parameters: pair terms and (beta, eta) from entry
 *    (t_i, t_j, t_j); zeta terms and the cutoff applied to r_ik from entry
 *    (t_i, t_j, t_k);
 *  - a bond with zeta = 0 has b = 1 and db/dzeta = 0.
 * The virial is W_ab = sum over every pair and triplet force term of
 * r_a F_b, with r the relative vector from the centre atom i.
 *
 * Minimum image: per axis s = rint(d / L) (IEEE division, ties to even),
 * d' = fma(-s, L, d); r^2 = fma(dz, dz, fma(dy, dy, dx*dx)).  The neighbour
 * list holds every j != i with r^2 < (cutoff + skin)^2, rows sorted by j.
 * Build with -ffp-contract=off so that the predicate is exactly this
 * sequence of roundings.
 *
 * Parameter table layout: ntypes^3 entries, entry (ti, tj, tk) at
 * ((ti*nt + tj)*nt + tk), 14 doubles each in the order
 * A, B, lambda1, lambda2, lambda3, beta, eta, c, d, h, gamma, R, D, m.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { OA = 0, OB, OL1, OL2, OL3, OBETA, OETA, OC, OD, OH, OGAMMA, OR, ODC, OM, ONP };

static const double ORACLE_PI = 3.14159265358979323846;

/* ---------------------------------------------------------------- geometry */

static void min_image(const double *xi, const double *xj, const double *L, double d[3])
{
    for (int a = 0; a < 3; ++a) {
        double t = xj[a] - xi[a];
        double s = rint(t / L[a]);
        d[a] = fma(-s, L[a], t);
    }
}

static double norm2(const double d[3])
{
    return fma(d[2], d[2], fma(d[1], d[1], d[0] * d[0]));
}

/* ------------------------------------------------------- neighbour lists */

/* Brute force O(N^2): the definition.  Returns the number of entries; the
 * arrays are filled only when that number fits in cap. */
int64_t oracle_neighbors_brute(int64_t n, const double *pos, const double *box,
                               double rcut, int64_t *offsets, int32_t *idx, int64_t cap)
{
    const double rc2 = rcut * rcut;
    int64_t total = 0;
    for (int64_t i = 0; i < n; ++i) {
        offsets[i] = total;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3];
            min_image(pos + 3 * i, pos + 3 * j, box, d);
            if (norm2(d) < rc2) {
                if (total < cap) idx[total] = (int32_t)j;
                ++total;
            }
        }
    }
    offsets[n] = total;
    return total;
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Cell-list version for large N.  Cells are at least rcut*(1+1e-10) wide, so
 * every pair within rcut lies in the same or an adjacent cell; rows are
 * sorted afterwards.  Must equal oracle_neighbors_brute exactly. */
int64_t oracle_neighbors_cell(int64_t n, const double *pos, const double *box,
                              double rcut, int64_t *offsets, int32_t *idx, int64_t cap)
{
    const double rc2 = rcut * rcut;
    int nc[3];
    for (int a = 0; a < 3; ++a) {
        nc[a] = (int)floor(box[a] / (rcut * (1.0 + 1e-10)));
        if (nc[a] < 1) nc[a] = 1;
    }
    const int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    int64_t *head = malloc(sizeof(int64_t) * (size_t)(ncell + 1));
    int64_t *cell_of = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t *sorted = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t *fill = malloc(sizeof(int64_t) * (size_t)(ncell + 1));
    memset(head, 0, sizeof(int64_t) * (size_t)(ncell + 1));
    for (int64_t i = 0; i < n; ++i) {
        int c[3];
        for (int a = 0; a < 3; ++a) {
            double u = pos[3 * i + a] - box[a] * floor(pos[3 * i + a] / box[a]);
            int ci = (int)floor(u / (box[a] / nc[a]));
            if (ci < 0) ci = 0;
            if (ci >= nc[a]) ci = nc[a] - 1;
            c[a] = ci;
        }
        cell_of[i] = ((int64_t)c[0] * nc[1] + c[1]) * nc[2] + c[2];
        head[cell_of[i] + 1]++;
    }
    for (int64_t c = 0; c < ncell; ++c) head[c + 1] += head[c];
    memcpy(fill, head, sizeof(int64_t) * (size_t)(ncell + 1));
    for (int64_t i = 0; i < n; ++i) sorted[fill[cell_of[i]]++] = i;

    int64_t total = 0;
    for (int64_t i = 0; i < n; ++i) {
        offsets[i] = total;
        int64_t row0 = total;
        int64_t ci = cell_of[i];
        int c[3] = { (int)(ci / ((int64_t)nc[1] * nc[2])), (int)((ci / nc[2]) % nc[1]), (int)(ci % nc[2]) };
        /* unique neighbouring cells per axis */
        int off[3][3], noff[3];
        for (int a = 0; a < 3; ++a) {
            if (nc[a] >= 3) { off[a][0] = -1; off[a][1] = 0; off[a][2] = 1; noff[a] = 3; }
            else if (nc[a] == 2) { off[a][0] = 0; off[a][1] = 1; noff[a] = 2; }
            else { off[a][0] = 0; noff[a] = 1; }
        }
        for (int ox = 0; ox < noff[0]; ++ox)
        for (int oy = 0; oy < noff[1]; ++oy)
        for (int oz = 0; oz < noff[2]; ++oz) {
            int x = (c[0] + off[0][ox] + nc[0]) % nc[0];
            int y = (c[1] + off[1][oy] + nc[1]) % nc[1];
            int z = (c[2] + off[2][oz] + nc[2]) % nc[2];
            int64_t cc = ((int64_t)x * nc[1] + y) * nc[2] + z;
            for (int64_t s = head[cc]; s < head[cc + 1]; ++s) {
                int64_t j = sorted[s];
                if (j == i) continue;
                double d[3];
                min_image(pos + 3 * i, pos + 3 * j, box, d);
                if (norm2(d) < rc2) {
                    if (total < cap) idx[total] = (int32_t)j;
                    ++total;
                }
            }
        }
        if (total <= cap) qsort(idx + row0, (size_t)(total - row0), sizeof(int32_t), cmp_i32);
    }
    offsets[n] = total;
    free(head); free(cell_of); free(sorted); free(fill);
    return total;
}

/* --------------------------------------------------- functional forms */

/* In the switching zone f_C = 1/2 - 1/2 sin(pi/2 (r-R)/D) is evaluated as
 * sin^2(y), y = pi/4 (R+D-r)/D (the half-angle identity 1 - sin x =
 * 2 sin^2(pi/4 - x/2)): the same function, without the cancellation of
 * 1 - sin x near the cutoff, where f_C of a third atom is tiny but
 * dV/dzeta ~ zeta^(eta-1) keeps its force term finite (the literal form
 * loses all its digits within 1e-8 A of R + D).  f_C' = -pi/(4D) sin(2y). */
static void cutoff_fn(double r, const double *p, double *fc, double *dfc)
{
    double R = p[OR], D = p[ODC];
    if (r < R - D) { *fc = 1.0; *dfc = 0.0; }
    else if (r < R + D) {
        double y = ORACLE_PI / 4.0 * ((R + D) - r) / D;
        double s = sin(y);
        *fc = s * s;
        *dfc = -ORACLE_PI / (4.0 * D) * sin(2.0 * y);
    } else { *fc = 0.0; *dfc = 0.0; }
}

static double g_fn(double costh, const double *p)
{
    double c2 = p[OC] * p[OC], d2 = p[OD] * p[OD], t = costh - p[OH];
    return p[OGAMMA] * (1.0 + c2 / d2 - c2 / (d2 + t * t));
}

static double dg_fn(double costh, const double *p)
{
    double c2 = p[OC] * p[OC], d2 = p[OD] * p[OD], t = costh - p[OH];
    double q = d2 + t * t;
    return p[OGAMMA] * c2 * 2.0 * t / (q * q);
}

/* exp((lambda3 (rij - rik))^m) and its derivative with respect to rij */
static void exp_fn(double rij, double rik, const double *p, double *e, double *de)
{
    double l3 = p[OL3], dr = rij - rik;
    if ((int)p[OM] == 3) {
        double arg = pow(l3 * dr, 3.0);
        *e = exp(arg);
        *de = 3.0 * l3 * l3 * l3 * dr * dr * (*e);
    } else {
        *e = exp(l3 * dr);
        *de = l3 * (*e);
    }
}

/* zeta(i,j,k) and its gradients with respect to x_j and x_k */
static double zeta_term(const double *p, double rij, const double dij[3],
                        double rik, const double dik[3], double gj[3], double gk[3])
{
    double cos_t = (dij[0] * dik[0] + dij[1] * dik[1] + dij[2] * dik[2]) / (rij * rik);
    double fc, dfc, e, de;
    cutoff_fn(rik, p, &fc, &dfc);
    exp_fn(rij, rik, p, &e, &de);
    double g = g_fn(cos_t, p), dg = dg_fn(cos_t, p);
    if (gj) {
        for (int a = 0; a < 3; ++a) {
            double uij = dij[a] / rij, uik = dik[a] / rik;
            double dcos_j = (uik - cos_t * uij) / rij;
            double dcos_k = (uij - cos_t * uik) / rik;
            gj[a] = fc * dg * dcos_j * e + fc * g * de * uij;
            gk[a] = dfc * uik * g * e + fc * dg * dcos_k * e - fc * g * de * uik;
        }
    }
    return fc * g * e;
}

/* ------------------------------------------------ energy and its gradient */

/* E of Eq. (1) and F = -dE/dx by the chain rule, centre by centre, summing
 * the contributions of centre atoms i in [i0, i1).  For a centre i, the
 * displacements of its list entries are formed once.  For each bond (i, j)
 * within the cutoff of entry (t_i, t_j, t_j), the terms of zeta_ij (Eq. 3)
 * over the third atoms k are formed together with their gradients with
 * respect to x_j and x_k; b_ij (Eq. 2) and the bond energy
 * V_ij = 1/2 f_C [f_R + b_ij f_A] follow, and dE/dx takes
 *   dV/dr_ij u_ij + dV/dzeta_ij sum_k dzeta(i,j,k)/dx_j   on j,
 *   dV/dzeta_ij dzeta(i,j,k)/dx_k                        on each k,
 * and minus their sum on i (V depends on positions relative to x_i only).
 * The virial sums r (x) F over these terms, r the vector from x_i.
 * forces (n x 3) and virial (6: xx yy zz xy xz yz) are overwritten.
 * Returns 0, -1 on a type out of range, -2 when out of memory. */
int oracle_compute(int64_t n, const double *pos, const int32_t *types, const double *box,
                   const double *table, int32_t nt, const int64_t *offsets,
                   const int32_t *idx, int64_t i0, int64_t i1, int32_t nthreads,
                   double *energy, double *forces, double *virial)
{
    for (int64_t i = 0; i < n; ++i)
        if (types[i] < 0 || types[i] >= nt) return -1;
    if (i0 < 0) i0 = 0;
    if (i1 > n) i1 = n;
    int64_t maxrow = 1;
    for (int64_t i = i0; i < i1; ++i)
        if (offsets[i + 1] - offsets[i] > maxrow) maxrow = offsets[i + 1] - offsets[i];
    int nth = nthreads > 0 ? nthreads : 1;
#ifdef _OPENMP
    if (nth > omp_get_max_threads()) nth = omp_get_max_threads();
#else
    nth = 1;
#endif
    if (nth > 64) nth = 64;
    double *fpriv = calloc((size_t)nth * (size_t)(3 * n > 0 ? 3 * n : 1), sizeof(double));
    /* per thread: each entry's displacement (3), r^2 and dE/dx_k (3) */
    double *scratch = malloc((size_t)nth * (size_t)maxrow * 7 * sizeof(double));
    if (!fpriv || !scratch) {
        free(fpriv);
        free(scratch);
        return -2;
    }
    double epriv[64] = {0}, wpriv[64][6];
    memset(wpriv, 0, sizeof(wpriv));

#ifdef _OPENMP
#pragma omp parallel num_threads(nth)
#endif
    {
#ifdef _OPENMP
        int tid = omp_get_thread_num();
#else
        int tid = 0;
#endif
        double *F = fpriv + (size_t)tid * 3 * (size_t)n;
        double *dsp = scratch + (size_t)tid * (size_t)maxrow * 7;   /* displacements */
        double *rsq = dsp + 3 * maxrow;                               /* r^2 */
        double *gk = rsq + maxrow;                                    /* dE/dx_k of one bond */
        double E = 0.0, W[6] = {0, 0, 0, 0, 0, 0};
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 256)
#endif
        for (int64_t i = i0; i < i1; ++i) {
            const int ti = types[i];
            const int64_t e0 = offsets[i], m = offsets[i + 1] - offsets[i];
            for (int64_t q = 0; q < m; ++q) {
                min_image(pos + 3 * i, pos + 3 * idx[e0 + q], box, dsp + 3 * q);
                rsq[q] = norm2(dsp + 3 * q);
            }
            for (int64_t jq = 0; jq < m; ++jq) {
                const int64_t j = idx[e0 + jq];
                const int tj = types[j];
                const double *pij = table + (size_t)((ti * nt + tj) * nt + tj) * ONP;
                const double cut = pij[OR] + pij[ODC];
                if (!(rsq[jq] < cut * cut)) continue;
                const double *dij = dsp + 3 * jq;
                const double rij = sqrt(rsq[jq]);

                /* zeta_ij, sum_k dzeta/dx_j, and each dzeta/dx_k */
                double zeta = 0.0, gj_sum[3] = {0, 0, 0};
                for (int64_t kq = 0; kq < m; ++kq) {
                    gk[3 * kq] = gk[3 * kq + 1] = gk[3 * kq + 2] = 0.0;
                    if (kq == jq) continue;
                    const double *pk = table + (size_t)((ti * nt + tj) * nt + types[idx[e0 + kq]]) * ONP;
                    const double cutk = pk[OR] + pk[ODC];
                    if (!(rsq[kq] < cutk * cutk)) continue;
                    double gj[3];
                    zeta += zeta_term(pk, rij, dij, sqrt(rsq[kq]), dsp + 3 * kq, gj, gk + 3 * kq);
                    for (int a = 0; a < 3; ++a) gj_sum[a] += gj[a];
                }

                /* Eq. (1)-(2): the bond's energy and its derivatives */
                double fc, dfc;
                cutoff_fn(rij, pij, &fc, &dfc);
                const double fr = pij[OA] * exp(-pij[OL1] * rij), dfr = -pij[OL1] * fr;
                const double fa = -pij[OB] * exp(-pij[OL2] * rij), dfa = -pij[OL2] * fa;
                const double beta = pij[OBETA], eta = pij[OETA];
                const double x = pow(beta * zeta, eta);
                const double b = pow(1.0 + x, -1.0 / (2.0 * eta));
                double db = 0.0;
                if (zeta > 0.0)
                    db = -0.5 * pow(1.0 + x, -1.0 / (2.0 * eta) - 1.0) * pow(beta, eta) * pow(zeta, eta - 1.0);
                E += 0.5 * fc * (fr + b * fa);
                const double dVdr = 0.5 * (dfc * (fr + b * fa) + fc * (dfr + b * dfa));
                const double dVdz = 0.5 * fc * fa * db;

                /* dE/dx on j and on each k; minus their sum on i */
                double dEj[3], dEi[3];
                for (int a = 0; a < 3; ++a) {
                    dEj[a] = dVdr * dij[a] / rij + dVdz * gj_sum[a];
                    dEi[a] = -dEj[a];
                    F[3 * j + a] -= dEj[a];
                }
                W[0] -= dij[0] * dEj[0];
                W[1] -= dij[1] * dEj[1];
                W[2] -= dij[2] * dEj[2];
                W[3] -= dij[0] * dEj[1];
                W[4] -= dij[0] * dEj[2];
                W[5] -= dij[1] * dEj[2];
                if (dVdz != 0.0) {
                    for (int64_t kq = 0; kq < m; ++kq) {
                        const double *g = gk + 3 * kq;
                        if (g[0] == 0.0 && g[1] == 0.0 && g[2] == 0.0) continue;
                        const int64_t k = idx[e0 + kq];
                        const double *dik = dsp + 3 * kq;
                        double dEk[3];
                        for (int a = 0; a < 3; ++a) {
                            dEk[a] = dVdz * g[a];
                            dEi[a] -= dEk[a];
                            F[3 * k + a] -= dEk[a];
                        }
                        W[0] -= dik[0] * dEk[0];
                        W[1] -= dik[1] * dEk[1];
                        W[2] -= dik[2] * dEk[2];
                        W[3] -= dik[0] * dEk[1];
                        W[4] -= dik[0] * dEk[2];
                        W[5] -= dik[1] * dEk[2];
                    }
                }
                for (int a = 0; a < 3; ++a) F[3 * i + a] -= dEi[a];
            }
        }
        epriv[tid] = E;
        for (int c = 0; c < 6; ++c) wpriv[tid][c] = W[c];
    }

    double E = 0.0;
    for (int c = 0; c < 6; ++c) virial[c] = 0.0;
    for (int t = 0; t < nth; ++t) {
        E += epriv[t];
        for (int c = 0; c < 6; ++c) virial[c] += wpriv[t][c];
    }
    for (int64_t q = 0; q < 3 * n; ++q) {
        double s = 0.0;
        for (int t = 0; t < nth; ++t) s += fpriv[(size_t)t * 3 * (size_t)n + (size_t)q];
        forces[q] = s;
    }
    *energy = E;
    free(fpriv);
    free(scratch);
    return 0;
}

/* Work counts of one evaluation: list entries S, in-cutoff ordered pairs P,
 * and ordered triplets T (i; j, k in cutoff, k != j) over centres [i0, i1). */
void oracle_counts(int64_t n, const double *pos, const int32_t *types, const double *box,
                   const double *table, int32_t nt, const int64_t *offsets,
                   const int32_t *idx, int64_t i0, int64_t i1, int64_t out[3])
{
    int64_t S = 0, P = 0, T = 0;
    (void)n;
    for (int64_t i = i0; i < i1; ++i) {
        int ti = types[i];
        S += offsets[i + 1] - offsets[i];
        for (int64_t jj = offsets[i]; jj < offsets[i + 1]; ++jj) {
            int64_t j = idx[jj];
            int tj = types[j];
            const double *pij = table + (size_t)((ti * nt + tj) * nt + tj) * ONP;
            double dij[3];
            min_image(pos + 3 * i, pos + 3 * j, box, dij);
            double cut = pij[OR] + pij[ODC];
            if (!(norm2(dij) < cut * cut)) continue;
            ++P;
            for (int64_t kk = offsets[i]; kk < offsets[i + 1]; ++kk) {
                int64_t k = idx[kk];
                if (k == j) continue;
                const double *pk = table + (size_t)((ti * nt + tj) * nt + types[k]) * ONP;
                double dik[3];
                min_image(pos + 3 * i, pos + 3 * k, box, dik);
                double cutk = pk[OR] + pk[ODC];
                if (norm2(dik) < cutk * cutk) ++T;
            }
        }
    }
    out[0] = S; out[1] = P; out[2] = T;
}
