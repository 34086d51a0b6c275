/*
 * CPU oracle for the strong-form spectral-element volume term of the dry
 * Euler equations (Klöckner, Wilcox, Warburton, "Array Program Transformation
 * with Loo.py by Example: High-Order Finite Elements", ARRAY'16, Sec. 2).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker the HIP path is compared
 * against.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it.  It shares no code, header or table with the HIP
 * library, and the library never calls it.
 *
 * Plain FP64 loops, strict IEEE (built with -O2 -ffp-contract=off, no
 * fast-math), OpenMP over elements only.  The flux is evaluated once per node
 * (Cartesian physical flux f_ab), then Eq. (volterm) is summed exactly as
 * written: over the line index n and the flux direction a, separately for the
 * three reference directions.
 *
 * Array layouts (all row-major, element outermost):
 *   D[i*Nq + n]            = l_n'(xi_i)
 *   geo[e][10][Nq^3]       slot 3*d + a = g_{a d} (a, d = 0..2), slot 9 = 1/J
 *   q, rhs[e][5][Nq^3]     fields rho, U1, U2, U3, Theta
 *   rho_ref, theta_ref[e][Nq^3]  (both NULL, or both given)
 *   node index m = i + Nq*j + Nq^2*k   (i, j, k along r, s, t)
 *
 * Readings taken where the paper is silent or inconsistent:
 *   - sign: the volume term is -(1/J) * sum(...), as the listed r/s kernels
 *     subtract from rhsq and as the PDE dq/dt = -div f demands (Eq. (volterm)
 *     prints "+");
 *   - g_{ad} = J * dxi_d/dx_a sits inside the sum at the line node n, 1/J is
 *     taken at the output node (the listed kernels read geo slot 10 at (i,j,k));
 *   - gravity (left out by the paper) enters as the source -grav*(rho-rho_ref)
 *     on U3 only, with x_3 vertical;
 *   - with a reference state the pressure in the flux is the perturbation
 *     p - p_ref, p_ref = EOS(Theta_ref); without one it is the full p.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Equation of state, Sec. 2: p = p0 (R Theta / p0)^gamma. */
static double eos_pressure(double theta, double p0, double gamma, double R)
{
    return p0 * pow(R * theta / p0, gamma);
}

/* Flux column f_a(q) of equation set 2C (Sec. 2): f[a][b] for direction
 * a = 0..2 and field b < nf, with nf = 5 (rho, U1, U2, U3, Theta) or 8 (plus
 * the passive tracers Q1, Q2, Q3):
 *   f_a = [U_a, U_a U_1/rho + delta_a1 p, U_a U_2/rho + delta_a2 p,
 *          U_a U_3/rho + delta_a3 p, U_a Theta/rho, U_a Q_i/rho]. */
#define MAXF 8
static void physical_flux(const double* qn, int nf, double p, double f[3][MAXF])
{
    const double rho = qn[0];
    for (int a = 0; a < 3; ++a) {
        const double Ua = qn[1 + a];
        f[a][0] = Ua;
        for (int c = 0; c < 3; ++c)
            f[a][1 + c] = Ua * qn[1 + c] / rho + (a == c ? p : 0.0);
        for (int b = 4; b < nf; ++b)
            f[a][b] = Ua * qn[b] / rho;
    }
}

/* Derivative of the flux column with respect to the state, obtained by
 * differentiating the expressions above term by term:
 * J[a][b][c] = d f_ab / d q_c, q = (rho, U1, U2, U3, Theta), with
 * dp/dTheta = gamma p / Theta from the EOS. */
static void flux_jacobian(const double qn[5], double dp_dtheta, double J[3][5][5])
{
    const double rho = qn[0];
    memset(J, 0, sizeof(double) * 3 * 5 * 5);
    for (int a = 0; a < 3; ++a) {
        const double Ua = qn[1 + a];
        /* f_a0 = U_a */
        J[a][0][1 + a] = 1.0;
        /* f_a(1+e) = U_a U_e / rho + delta_ae p */
        for (int e = 0; e < 3; ++e) {
            const double Ue = qn[1 + e];
            J[a][1 + e][0] = -Ua * Ue / (rho * rho);
            J[a][1 + e][1 + a] += Ue / rho;
            J[a][1 + e][1 + e] += Ua / rho;
            if (a == e)
                J[a][1 + e][4] = dp_dtheta;
        }
        /* f_a4 = U_a Theta / rho */
        J[a][4][0] = -Ua * qn[4] / (rho * rho);
        J[a][4][1 + a] = qn[4] / rho;
        J[a][4][4] = Ua / rho;
    }
}

int sem_oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void sem_oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/*
 * Volume term, Eq. (volterm), plus the gravity source:
 *   v_b(i,j,k) = -(1/J(i,j,k)) * sum_{n,a} [ D[i][n] g_a1(n,j,k) f_ab(n,j,k)
 *                                          + D[j][n] g_a2(i,n,k) f_ab(i,n,k)
 *                                          + D[k][n] g_a3(i,j,n) f_ab(i,j,n) ]
 *   v_U3 += -grav * (rho - rho_ref)
 * for nf = 5 or 8 fields (q, rhs [e][nf][Nq^3]).  `dirs` selects which of the
 * three sums enter (bit 0 = r, bit 1 = s, bit 2 = t): the paper's benchmark
 * kernel fuses the r and s terms only (dirs = 3).  Elements [e0, e1) are
 * evaluated; rhs is indexed like q.  accumulate != 0 adds to rhs instead of
 * overwriting (the listed kernels' rhsq update).
 */
void sem_oracle_volume_rhs_ext(int64_t e0, int64_t e1, int32_t Nq, int32_t nf, uint32_t dirs,
                               const double* D, const double* geo, const double* q,
                               const double* rho_ref, const double* theta_ref,
                               double p0, double gamma, double R, double grav,
                               double* rhs, int32_t accumulate)
{
    const int64_t M = (int64_t)Nq * Nq * Nq;
    const int use_r = (dirs & 1u) != 0, use_s = (dirs & 2u) != 0, use_t = (dirs & 4u) != 0;
#pragma omp parallel
    {
        double* f = (double*)malloc(sizeof(double) * (size_t)M * 3 * MAXF);
#pragma omp for schedule(static)
        for (int64_t e = e0; e < e1; ++e) {
            const double* qe = q + e * nf * M;
            const double* ge = geo + e * 10 * M;
            double* re = rhs + e * nf * M;
            /* pointwise: pressure (perturbation if a reference is given) and
             * the physical flux at every node, stored f[m][a][b] */
            for (int64_t m = 0; m < M; ++m) {
                double qn[MAXF];
                for (int b = 0; b < nf; ++b)
                    qn[b] = qe[b * M + m];
                double p = eos_pressure(qn[4], p0, gamma, R);
                if (theta_ref)
                    p -= eos_pressure(theta_ref[e * M + m], p0, gamma, R);
                physical_flux(qn, nf, p, (double(*)[MAXF])(f + m * 3 * MAXF));
            }
#define G(a, d, node) ge[(3 * (d) + (a)) * M + (node)]
#define F(node, a, b) f[(node) * 3 * MAXF + (a) * MAXF + (b)]
            for (int k = 0; k < Nq; ++k)
                for (int j = 0; j < Nq; ++j)
                    for (int i = 0; i < Nq; ++i) {
                        const int64_t m = i + (int64_t)Nq * j + (int64_t)Nq * Nq * k;
                        const double Jinv = ge[9 * M + m];
                        for (int b = 0; b < nf; ++b) {
                            double sr = 0.0, ss = 0.0, st = 0.0;
                            for (int n = 0; n < Nq; ++n)
                                for (int a = 0; a < 3; ++a) {
                                    const int64_t nr = n + (int64_t)Nq * j + (int64_t)Nq * Nq * k;
                                    const int64_t ns = i + (int64_t)Nq * n + (int64_t)Nq * Nq * k;
                                    const int64_t nt = i + (int64_t)Nq * j + (int64_t)Nq * Nq * n;
                                    sr += D[i * Nq + n] * G(a, 0, nr) * F(nr, a, b);
                                    ss += D[j * Nq + n] * G(a, 1, ns) * F(ns, a, b);
                                    st += D[k * Nq + n] * G(a, 2, nt) * F(nt, a, b);
                                }
                            double v = -Jinv * ((use_r ? sr : 0.0) + (use_s ? ss : 0.0) +
                                                (use_t ? st : 0.0));
                            if (b == 3) {
                                const double rr = rho_ref ? rho_ref[e * M + m] : 0.0;
                                v += -grav * (qe[m] - rr);
                            }
                            re[b * M + m] = accumulate ? re[b * M + m] + v : v;
                        }
                    }
#undef G
#undef F
        }
        free(f);
    }
}

/* The five-field volume term with all three directions (the operation the
 * library's sem_volume_rhs computes). */
void sem_oracle_volume_rhs(int64_t e0, int64_t e1, int32_t Nq, const double* D,
                           const double* geo, const double* q,
                           const double* rho_ref, const double* theta_ref,
                           double p0, double gamma, double R, double grav,
                           double* rhs, int32_t accumulate)
{
    sem_oracle_volume_rhs_ext(e0, e1, Nq, 5, 7u, D, geo, q, rho_ref, theta_ref, p0, gamma, R, grav,
                              rhs, accumulate);
}

/*
 * Vector-Jacobian product of the volume term with respect to the state:
 *   mu_c(y) = sum_{x,b} lambda_b(x) d v_b(x) / d q_c(y).
 * Since v_b(x) = -(1/J(x)) sum_d sum_y' Dd[x][y'] sum_a g_ad(y') f_ab(q(y'))
 * + source, this is
 *   w_b(x)    = -(1/J(x)) lambda_b(x)
 *   G^d_b(y)  = sum_x Dd[x][y] w_b(x)     (transposed line contraction)
 *   H_ab(y)   = sum_d g_ad(y) G^d_b(y)
 *   mu_c(y)   = sum_{a,b} H_ab(y) d f_ab/d q_c (y)  - grav lambda_U3(y) [c = rho]
 * The reference state drops out: d(p - p_ref)/dTheta = dp/dTheta and
 * d(rho - rho_ref)/drho = 1.
 */
void sem_oracle_volume_rhs_adjoint(int64_t e0, int64_t e1, int32_t Nq, const double* D,
                                   const double* geo, const double* q,
                                   double p0, double gamma, double R, double grav,
                                   const double* lambda, double* mu, int32_t accumulate)
{
    const int64_t M = (int64_t)Nq * Nq * Nq;
#pragma omp parallel
    {
        double* w = (double*)malloc(sizeof(double) * (size_t)M * 5);
        double* G = (double*)malloc(sizeof(double) * (size_t)M * 15);
#pragma omp for schedule(static)
        for (int64_t e = e0; e < e1; ++e) {
            const double* qe = q + e * 5 * M;
            const double* ge = geo + e * 10 * M;
            const double* le = lambda + e * 5 * M;
            double* me = mu + e * 5 * M;
            for (int64_t m = 0; m < M; ++m)
                for (int b = 0; b < 5; ++b)
                    w[m * 5 + b] = -ge[9 * M + m] * le[b * M + m];
            /* G[y][d][b] */
            memset(G, 0, sizeof(double) * (size_t)M * 15);
            for (int k = 0; k < Nq; ++k)
                for (int j = 0; j < Nq; ++j)
                    for (int i = 0; i < Nq; ++i) {
                        const int64_t x = i + (int64_t)Nq * j + (int64_t)Nq * Nq * k;
                        for (int n = 0; n < Nq; ++n) {
                            const int64_t yr = n + (int64_t)Nq * j + (int64_t)Nq * Nq * k;
                            const int64_t ys = i + (int64_t)Nq * n + (int64_t)Nq * Nq * k;
                            const int64_t yt = i + (int64_t)Nq * j + (int64_t)Nq * Nq * n;
                            for (int b = 0; b < 5; ++b) {
                                G[yr * 15 + 0 * 5 + b] += D[i * Nq + n] * w[x * 5 + b];
                                G[ys * 15 + 1 * 5 + b] += D[j * Nq + n] * w[x * 5 + b];
                                G[yt * 15 + 2 * 5 + b] += D[k * Nq + n] * w[x * 5 + b];
                            }
                        }
                    }
            for (int64_t y = 0; y < M; ++y) {
                double qn[5];
                for (int b = 0; b < 5; ++b)
                    qn[b] = qe[b * M + y];
                const double p = eos_pressure(qn[4], p0, gamma, R);
                double Jf[3][5][5];
                flux_jacobian(qn, gamma * p / qn[4], Jf);
                double H[3][5];
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 5; ++b) {
                        double s = 0.0;
                        for (int d = 0; d < 3; ++d)
                            s += ge[(3 * d + a) * M + y] * G[y * 15 + d * 5 + b];
                        H[a][b] = s;
                    }
                for (int c = 0; c < 5; ++c) {
                    double s = 0.0;
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 5; ++b)
                            s += H[a][b] * Jf[a][b][c];
                    if (c == 0)
                        s += -grav * le[3 * M + y];
                    me[c * M + y] = accumulate ? me[c * M + y] + s : s;
                }
            }
        }
        free(w);
        free(G);
    }
}
