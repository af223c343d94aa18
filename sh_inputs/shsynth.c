/*
 * Seeded test-field synthesis: sums of real, orthonormal spherical harmonics
 * evaluated on the half-shifted colatitude grid theta_j = (j + 1/2) pi / m.
 *
 * This file produces INPUTS only.  It contains no part of the Poisson method
 * (no doubling, no transforms of the solver, no linear solves).  It returns,
 * for every azimuthal order M and every colatitude theta_j, the Legendre sums
 *
 *     A_M(theta_j) = w_M * sum_{l >= max(M,1)} c_{l,+M} Pbar_l^M(cos theta_j)
 *     B_M(theta_j) = w_M * sum_{l >= max(M,1)} c_{l,-M} Pbar_l^M(cos theta_j)
 *
 * with w_0 = 1, w_M = sqrt(2) for M > 0, so that the field is
 *     f(lambda, theta) = sum_M A_M(theta) cos(M lambda) + B_M(theta) sin(M lambda).
 * Pbar_l^M is the associated Legendre function normalised so that the real
 * harmonics have unit L2 norm on the sphere (no Condon-Shortley phase).
 *
 * Coefficient layout of one set: l = 1..L ascending, and for each l the
 * orders M = -l..l ascending; entry (l, M) sits at index l*l - 1 + (M + l).
 *
 * Recurrences (standard, fully normalised):
 *   Pbar_0^0 = 1/sqrt(4 pi)
 *   Pbar_M^M = sqrt((2M+1)/(2M)) sin(theta) Pbar_{M-1}^{M-1}
 *   Pbar_{M+1}^M = sqrt(2M+3) cos(theta) Pbar_M^M
 *   Pbar_l^M = a_lM (cos(theta) Pbar_{l-1}^M - b_lM Pbar_{l-2}^M),
 *     a_lM = sqrt((4l^2-1)/(l^2-M^2)), b_lM = sqrt(((l-1)^2-M^2)/(4(l-1)^2-1)).
 * Sectoral values (sin theta)^M fall far below the double range near the
 * poles for large M, while the recurrence in l later grows them back by up to
 * hundreds of orders of magnitude.  They are therefore carried as
 * value * 2^e with an integer exponent e (a multiple of 400, e <= 0).  The
 * recurrence runs on the scaled value; whenever the true value reaches 2^-600
 * it is converted back to an ordinary double (e = 0), and while it is smaller
 * a scaled value above 2^400 is renormalised by 2^-400.  Terms whose true value
 * stays below 2^-600 (about 1e-181) are left out of the sums.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Returns 0 on success, -1 on bad arguments, -2 on allocation failure.
 * A and B are [nsets][L+1][m] row-major (theta fastest). */
int sh_legendre_sums(int m, int L, int nsets, const double* coeffs,
                     double* A, double* B) {
    if (m < 1 || L < 0 || nsets < 1 || !coeffs || !A || !B) return -1;
    const int half = (m + 1) / 2;          /* theta_j for j < half lie in (0, pi/2] */
    const long ncoef = (long)(L + 1) * (L + 1) - 1;
    const double up = 0x1p400, down = 0x1p-400;
    double* x = (double*)malloc(sizeof(double) * half);
    double* s = (double*)malloc(sizeof(double) * half);
    double* pmm = (double*)malloc(sizeof(double) * (size_t)(L + 1) * half);
    int* pme = (int*)malloc(sizeof(int) * (size_t)(L + 1) * half);
    if (!x || !s || !pmm || !pme) { free(x); free(s); free(pmm); free(pme); return -2; }
    for (int j = 0; j < half; ++j) {
        double th = (j + 0.5) * M_PI / m;
        x[j] = cos(th);
        s[j] = sin(th);
    }
    /* Sectoral values Pbar_M^M(theta_j) = pmm * 2^pme: running product in M */
    for (int j = 0; j < half; ++j) { pmm[j] = 1.0 / sqrt(4.0 * M_PI); pme[j] = 0; }
    for (int M = 1; M <= L; ++M) {
        double f = sqrt((2.0 * M + 1.0) / (2.0 * M));
        double* cur = pmm + (size_t)M * half;
        const double* prv = pmm + (size_t)(M - 1) * half;
        int* ce = pme + (size_t)M * half;
        const int* pe = pme + (size_t)(M - 1) * half;
        for (int j = 0; j < half; ++j) {
            double v = f * s[j] * prv[j];
            int e = pe[j];
            if (v < down) { v *= up; e -= 400; }
            cur[j] = v;
            ce[j] = e;
        }
    }
    memset(A, 0, sizeof(double) * (size_t)nsets * (L + 1) * m);
    memset(B, 0, sizeof(double) * (size_t)nsets * (L + 1) * m);
    int failed = 0;
#pragma omp parallel
    {
        double* p0 = (double*)malloc(sizeof(double) * half);
        double* p1 = (double*)malloc(sizeof(double) * half);
        int* ex = (int*)malloc(sizeof(int) * half);
        double* acc = (double*)malloc(sizeof(double) * (size_t)4 * nsets * half);
        if (!p0 || !p1 || !ex || !acc) {
#pragma omp atomic write
            failed = 1;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int M = 0; M <= L; ++M) {
                memset(acc, 0, sizeof(double) * (size_t)4 * nsets * half);
                const double* pm = pmm + (size_t)M * half;
                const int* pe = pme + (size_t)M * half;
                /* the scaled entries form a prefix j < jz (sin theta grows with j) */
                int jz = 0;
                for (int j = 0; j < half; ++j) {
                    p0[j] = 0.0;
                    p1[j] = pm[j];
                    ex[j] = pe[j];
                    if (ex[j] < 0 && fabs(p1[j]) >= ldexp(1.0, -600 - ex[j])) {
                        p1[j] = ldexp(p1[j], ex[j]);
                        ex[j] = 0;
                    }
                    if (ex[j] < 0) jz = j + 1;
                }
                /* p1 holds Pbar_l^M (times 2^-ex) for the current l, p0 the previous l */
                for (int l = M; l <= L; ++l) {
                    double a = 0.0, b = 0.0;
                    if (l == M + 1) {
                        a = sqrt(2.0 * M + 3.0);
                    } else if (l > M + 1) {
                        double ll = (double)l, mm = (double)M;
                        a = sqrt((4.0 * ll * ll - 1.0) / (ll * ll - mm * mm));
                        b = sqrt(((ll - 1.0) * (ll - 1.0) - mm * mm) / (4.0 * (ll - 1.0) * (ll - 1.0) - 1.0));
                    }
                    if (l > M) {
                        for (int j = 0; j < jz; ++j) {
                            double nv = a * (x[j] * p1[j] - b * p0[j]);
                            p0[j] = p1[j];
                            p1[j] = nv;
                            if (ex[j] < 0) {
                                if (fabs(nv) > up) {
                                    p0[j] *= down;
                                    p1[j] *= down;
                                    ex[j] += 400;
                                }
                                if (ex[j] < 0 && fabs(p1[j]) >= ldexp(1.0, -600 - ex[j])) {
                                    p0[j] = ldexp(p0[j], ex[j]);
                                    p1[j] = ldexp(p1[j], ex[j]);
                                    ex[j] = 0;
                                }
                            }
                        }
                        for (int j = jz; j < half; ++j) {
                            double nv = a * (x[j] * p1[j] - b * p0[j]);
                            p0[j] = p1[j];
                            p1[j] = nv;
                        }
                    }
                    if (l == 0) continue; /* the l = 0 harmonic is never drawn */
                    int odd = (l + M) & 1;
                    for (int t = 0; t < nsets; ++t) {
                        const double* c = coeffs + (size_t)t * ncoef;
                        double cp = c[(long)l * l - 1 + (M + l)];
                        double cn = (M > 0) ? c[(long)l * l - 1 + (-M + l)] : 0.0;
                        double* ap = acc + ((size_t)(4 * t + 2 * 0 + odd)) * half;
                        double* an = acc + ((size_t)(4 * t + 2 * 1 + odd)) * half;
                        for (int j = 0; j < jz; ++j) {
                            if (ex[j] == 0) {
                                ap[j] += cp * p1[j];
                                an[j] += cn * p1[j];
                            }
                        }
                        for (int j = jz; j < half; ++j) {
                            ap[j] += cp * p1[j];
                            an[j] += cn * p1[j];
                        }
                    }
                }
                double w = (M == 0) ? 1.0 : sqrt(2.0);
                for (int t = 0; t < nsets; ++t) {
                    double* Ao = A + ((size_t)t * (L + 1) + M) * m;
                    double* Bo = B + ((size_t)t * (L + 1) + M) * m;
                    const double* ae = acc + (size_t)(4 * t + 0) * half;
                    const double* ao = acc + (size_t)(4 * t + 1) * half;
                    const double* be = acc + (size_t)(4 * t + 2) * half;
                    const double* bo = acc + (size_t)(4 * t + 3) * half;
                    for (int j = 0; j < half; ++j) {
                        /* theta_{m-1-j} = pi - theta_j: Pbar_l^M flips sign when l+M is odd */
                        Ao[j] = w * (ae[j] + ao[j]);
                        Bo[j] = w * (be[j] + bo[j]);
                        if (m - 1 - j != j) {
                            Ao[m - 1 - j] = w * (ae[j] - ao[j]);
                            Bo[m - 1 - j] = w * (be[j] - bo[j]);
                        }
                    }
                }
            }
        }
        free(p0); free(p1); free(ex); free(acc);
    }
    free(x); free(s); free(pmm); free(pme);
    return failed ? -2 : 0;
}
