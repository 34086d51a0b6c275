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
 *     p - p_ref, p_ref = EOS(Theta_ref); without one it is the full p;
 *   - the surface term s of dq/dt = v + s (Sec. 2 names it, the paper does
 *     not define it) is the strong-form discontinuous Galerkin face term on
 *     the same GLL nodes with a local Lax-Friedrichs (Rusanov) numerical flux;
 *     see sem_oracle_surface_rhs.
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

/*
 * Surface term s of the method-of-lines rate dq/dt = v(q) + s(q) (Sec. 2),
 * read as the strong-form discontinuous Galerkin face term on the GLL nodes
 * of the volume term (collocated quadrature), with a local Lax-Friedrichs
 * (Rusanov) numerical flux.
 *
 * Faces of element e: f = 2 d + side, d = 0, 1, 2 the reference direction
 * (r, s, t) and side 0 the face xi_d = -1, side 1 the face xi_d = +1.
 * nbr[e][f] is the element across face f.  Neighbours are conforming and
 * aligned: the neighbour's matching face is its face 2 d + (1 - side), and a
 * face node keeps its two tangential indices across the face (node
 * (0, j, k) of e meets node (N, j, k) of the element across its r = -1 face).
 * A neighbour index outside [0, Ne) marks a boundary face whose exterior
 * state equals the interior one, so that face adds nothing.
 *
 * At a node x of face (d, side), with sigma = -1 (side 0) or +1 (side 1):
 *   N      = sigma (g_0d, g_1d, g_2d)(x)      outward normal times area factor
 *   q-, q+ = the state of e at x, of the neighbour at its node of x
 *   p-, p+ = EOS pressure of q-, q+ (full pressure, for the sound speed)
 *   p'-, p'+ = the pressure in the flux: p- - p_ref-, p+ - p_ref+ with each
 *            side's own reference value (the volume term's pressure), or the
 *            full pressures when no reference state is given
 *   Fn(q, p') = sum_a N_a f_a(q, p')          normal flux
 *   c      = sqrt(gamma p / rho),  lambda = max(|u- . n| + c-, |u+ . n| + c+),
 *            n = N / |N|
 *   F*     = (Fn(q-, p'-) + Fn(q+, p'+)) / 2 - lambda |N| (q+ - q-) / 2
 *   s_b(x) += -(1/J(x)) / w_N * (F*_b - Fn_b(q-, p'-)),
 * w_N = 2 / (N (N + 1)) the GLL weight of the end nodes.  Nodes on an edge or
 * a corner collect the terms of each of their faces.  Where the reference
 * state is continuous across a face, p_ref cancels between F* and Fn(q-) and
 * s is the same with or without it; taking each side's own reference keeps
 * the two elements' numerical fluxes opposite where it is not (the z-periodic
 * faces of a stratified box), so that v + s stays conservative.
 *
 * Elements [e0, e1) are evaluated (rhs indexed like q); Ne bounds the
 * neighbour indices.  theta_ref [Ne][Nq^3] or NULL.  accumulate != 0 adds s to
 * rhs, else rhs = s (zero at interior nodes).
 */
void sem_oracle_surface_rhs(int64_t e0, int64_t e1, int64_t Ne, int32_t Nq, const int32_t* nbr,
                            const double* geo, const double* q, const double* theta_ref,
                            double p0, double gamma, double R, double* rhs, int32_t accumulate)
{
    const int64_t M = (int64_t)Nq * Nq * Nq;
    const int N = Nq - 1;
    const double wN = 2.0 / ((double)N * (N + 1));
    const int64_t stride[3] = {1, Nq, (int64_t)Nq * Nq};
#pragma omp parallel
    {
        double* sacc = (double*)malloc(sizeof(double) * (size_t)M * 5);
#pragma omp for schedule(static)
        for (int64_t e = e0; e < e1; ++e) {
            const double* qe = q + e * 5 * M;
            const double* ge = geo + e * 10 * M;
            memset(sacc, 0, sizeof(double) * (size_t)M * 5);
            for (int f = 0; f < 6; ++f) {
                const int d = f / 2, side = f % 2;
                const double sigma = side ? 1.0 : -1.0;
                const int64_t en = nbr[e * 6 + f];
                const int boundary = en < 0 || en >= Ne;
                /* the two tangential directions of the face */
                const int da = d == 0 ? 1 : 0, db = d == 2 ? 1 : 2;
                for (int b2 = 0; b2 < Nq; ++b2)
                    for (int a2 = 0; a2 < Nq; ++a2) {
                        const int64_t m = (side ? N : 0) * stride[d] + a2 * stride[da] +
                                          b2 * stride[db];
                        const int64_t mp = (side ? 0 : N) * stride[d] + a2 * stride[da] +
                                           b2 * stride[db];
                        double qm[5], qp[5];
                        for (int c = 0; c < 5; ++c) {
                            qm[c] = qe[c * M + m];
                            qp[c] = boundary ? qm[c] : q[en * 5 * M + c * M + mp];
                        }
                        double prm = 0.0, prp = 0.0;   /* reference pressures */
                        if (theta_ref) {
                            prm = eos_pressure(theta_ref[e * M + m], p0, gamma, R);
                            prp = boundary ? prm
                                           : eos_pressure(theta_ref[en * M + mp], p0, gamma, R);
                        }
                        double Nv[3], nn = 0.0;
                        for (int a = 0; a < 3; ++a) {
                            Nv[a] = sigma * ge[(3 * d + a) * M + m];
                            nn += Nv[a] * Nv[a];
                        }
                        nn = sqrt(nn);
                        const double pm = eos_pressure(qm[4], p0, gamma, R);
                        const double pp = eos_pressure(qp[4], p0, gamma, R);
                        double fm[3][MAXF], fp[3][MAXF];
                        physical_flux(qm, 5, pm - prm, fm);
                        physical_flux(qp, 5, pp - prp, fp);
                        const double unm = (Nv[0] * qm[1] + Nv[1] * qm[2] + Nv[2] * qm[3]) / (qm[0] * nn);
                        const double unp = (Nv[0] * qp[1] + Nv[1] * qp[2] + Nv[2] * qp[3]) / (qp[0] * nn);
                        const double lm = fabs(unm) + sqrt(gamma * pm / qm[0]);
                        const double lp = fabs(unp) + sqrt(gamma * pp / qp[0]);
                        const double lambda = lm > lp ? lm : lp;
                        const double jinv = ge[9 * M + m];
                        for (int c = 0; c < 5; ++c) {
                            double Fm = 0.0, Fp = 0.0;
                            for (int a = 0; a < 3; ++a) {
                                Fm += Nv[a] * fm[a][c];
                                Fp += Nv[a] * fp[a][c];
                            }
                            const double Fstar = 0.5 * (Fm + Fp) - 0.5 * lambda * nn * (qp[c] - qm[c]);
                            sacc[c * M + m] += -(jinv / wN) * (Fstar - Fm);
                        }
                    }
            }
            double* re = rhs + e * 5 * M;
            for (int64_t x = 0; x < 5 * M; ++x)
                re[x] = accumulate ? re[x] + sacc[x] : sacc[x];
        }
        free(sacc);
    }
}
