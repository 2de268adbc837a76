/*
 * lbm_oracle.c -- plain, slow FP64 CPU oracle for lattice-BGK with the
 * entropic equilibrium.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the reference the GPU library is checked
 * against.  The product path never includes, links or calls it: only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg load it.  It
 * shares no code, header, table or constant with the GPU library.
 *
 * Source: S. A. Hosseini and I. V. Karlin, "Entropic equilibrium for the lattice
 * Boltzmann method: Hydrodynamics and numerical properties", arXiv:2303.08163.
 *
 *   Sec. "Basic concepts"
 *       - the LBGK evolution equation f_i(r + c_i dt, t + dt) - f_i(r, t)
 *         = 2 beta (f_i^eq - f_i(r, t));
 *       - eq. (relaxation_frequency): beta = dt / (2 nu / varsigma^2 + dt);
 *       - varsigma = dr / (sqrt(3) dt);
 *       - the first-neighbour lattice: c in {-1, 0, 1}, 1-D weights
 *         {1/6, 2/3, 1/6}; 2-D and 3-D lattices as tensor products.
 *   Sec. "Discrete entropic equilibrium construction"
 *       - closed-form multipliers Z_alpha and X^{-1};
 *       - eq. (Entropic_isothermal_EDF): f_i^eq = w_i X^{-1} prod Z_alpha^{c_ia}.
 *   Sec. "Polynomial discrete equilibria"
 *       - eq. (Poly2_isothermal_EDF) and eq. (Product_isothermal_EDF); they
 *         serve the low-Mach checks and the alternative-equilibrium variants.
 *   Sec. "Navier-Stokes-level dynamics: dissipation", "1-D lattice"
 *       - eq. (entropic_bulk): the effective-viscosity factor A of the
 *         entropic equilibrium; eq. (LBGK_bulk): A of polynomial equilibria.
 *   Sec. "Correction of leading-order bulk viscosity error"
 *       - eq. (redefined_relaxation rate): beta = dt / (2 nu / (A varsigma^2) + dt);
 *       - eq. (redefined_relaxation rate_poly) for polynomial equilibria.
 *
 * Conventions (readings where the paper is silent):
 *   - lattice units dr = dt = 1, so varsigma^2 = 1/3;
 *   - nu is taken from the relaxation time tau as nu = varsigma^2 (tau - 1/2),
 *     which makes 2 beta = 1 / tau;
 *   - populations are ordered lexicographically over (c_x, c_y, c_z), x
 *     slowest; this ordering never leaves the oracle;
 *   - with the bulk correction, a node's A is min over axes of A(u_alpha)
 *     (corr_mode 1), or the product over axes (corr_mode 2); the paper derives
 *     A on a 1-D lattice only;
 *   - the streaming step pushes post-collision values to r + c_i on a periodic
 *     grid; fields are stored x fastest: node = x + nx (y + ny z);
 *   - the equilibrium is undefined for rho <= 0 or |u_alpha| >= 1; nodes that
 *     reach such a state are counted, nothing is clamped.
 *
 * Compiled with gcc -O2 -ffp-contract=off (no fast-math), optionally with
 * OpenMP over nodes; each node is computed independently, so the result does
 * not depend on the thread count.  The state, moments, relaxation and
 * streaming are IEEE double; the equilibrium's closed forms are evaluated in
 * extended precision and rounded once per population (see equilibrium_on).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_EQ_ENTROPIC 0
#define ORACLE_EQ_POLY2 1
#define ORACLE_EQ_PRODUCT 2

#define ORACLE_CORR_OFF 0
#define ORACLE_CORR_MIN 1
#define ORACLE_CORR_PRODUCT 2

/* Lattice sound speed squared, varsigma^2 = (dr / dt)^2 / 3 in lattice units. */
static const double CS2 = 1.0 / 3.0;

/* Sec. "Basic concepts": first-neighbour lattice in D dimensions.  Writes the
 * Q = 3^D velocities (3 ints each, unused components 0) and weights, which are
 * products of the 1-D weights {1/6, 2/3, 1/6}.  Returns Q, or -1 for bad D. */
int oracle_lattice(int D, int *c, double *w)
{
    static const double w1[3] = {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0}; /* c = -1, 0, 1 */
    if (D < 1 || D > 3)
        return -1;
    int Q = 1;
    for (int a = 0; a < D; a++)
        Q *= 3;
    for (int i = 0; i < Q; i++) {
        /* digit of axis a in base 3, axis 0 (x) most significant */
        int rem = i;
        int digits[3] = {1, 1, 1};
        for (int a = D - 1; a >= 0; a--) {
            digits[a] = rem % 3;
            rem /= 3;
        }
        double wi = 1.0;
        for (int a = 0; a < 3; a++) {
            int ca = (a < D) ? digits[a] - 1 : 0;
            c[3 * i + a] = ca;
            if (a < D)
                wi *= w1[digits[a]];
        }
        w[i] = wi;
    }
    return Q;
}

/* Equilibrium populations at one node.  kind selects
 *   ORACLE_EQ_ENTROPIC: eq. (Entropic_isothermal_EDF), built from the
 *       multipliers Z_alpha = (2 u_alpha + sqrt((u_alpha/varsigma)^2 + 1)) /
 *       (1 - u_alpha) and X^{-1} = rho prod_alpha (2 - sqrt((u_alpha/varsigma)^2
 *       + 1)), then f_i = w_i X^{-1} prod_alpha Z_alpha^{c_ia};
 *   ORACLE_EQ_POLY2: eq. (Poly2_isothermal_EDF);
 *   ORACLE_EQ_PRODUCT: eq. (Product_isothermal_EDF).
 * The closed forms are evaluated in extended precision (long double, 64-bit
 * significand on x86-64) and each f_i is rounded once to double.  The
 * equilibrium meets the mass and momentum constraints exactly (Sec. "Discrete
 * entropic equilibrium construction"); a double evaluation of the multiplier
 * form misses the momentum constraint by a few units in the last place with a
 * sign that stays the same from one step to the next, so under repeated
 * collisions it acts as a small spurious force and the velocity drifts
 * linearly in time.  One rounding per population keeps that below the
 * rounding of the state itself.
 * Returns 0, or 1 when (rho, u) lies outside the entropic equilibrium's domain
 * (rho <= 0, |u_alpha| >= 1, or a non-finite input); the values are still
 * written, whatever they evaluate to. */
typedef long double xreal;

static int equilibrium_on(int D, int Q, const int *c, const double *w, int kind, double rho,
                          const double *u, double *feq)
{
    const xreal cs2 = 1.0L / 3.0L;
    int bad = !(rho > 0.0) || !isfinite(rho);
    for (int a = 0; a < D; a++)
        if (!(fabs(u[a]) < 1.0))
            bad = 1;

    if (kind == ORACLE_EQ_ENTROPIC) {
        xreal Z[3], Xinv = rho;
        for (int a = 0; a < D; a++) {
            xreal ua = u[a];
            xreal root = sqrtl((ua * ua) / cs2 + 1.0L);
            Z[a] = (2.0L * ua + root) / (1.0L - ua);
            Xinv *= (2.0L - root);
        }
        for (int i = 0; i < Q; i++) {
            xreal prod = 1.0L;
            for (int a = 0; a < D; a++) {
                if (c[3 * i + a] == 1)
                    prod *= Z[a];
                else if (c[3 * i + a] == -1)
                    prod /= Z[a];
            }
            feq[i] = (double)((xreal)w[i] * Xinv * prod);
        }
    } else if (kind == ORACLE_EQ_POLY2) {
        xreal usq = 0.0L;
        for (int a = 0; a < D; a++)
            usq += (xreal)u[a] * u[a];
        for (int i = 0; i < Q; i++) {
            xreal cu = 0.0L;
            for (int a = 0; a < D; a++)
                cu += c[3 * i + a] * (xreal)u[a];
            feq[i] = (double)((xreal)w[i] * rho *
                              (1.0L + cu / cs2 + (cu * cu) / (2.0L * cs2 * cs2) - usq / (2.0L * cs2)));
        }
    } else if (kind == ORACLE_EQ_PRODUCT) {
        for (int i = 0; i < Q; i++) {
            xreal prod = rho;
            for (int a = 0; a < D; a++) {
                int ca = c[3 * i + a];
                xreal ua = u[a];
                if (ca == 0)
                    prod *= (1.0L - cs2 - ua * ua);
                else
                    prod *= (ca * ua + cs2 + ua * ua) / 2.0L;
            }
            feq[i] = (double)prod;
        }
    } else {
        return -1;
    }
    return bad;
}

int oracle_equilibrium(int D, int kind, double rho, const double *u, double *feq)
{
    int c[27 * 3];
    double w[27];
    int Q = oracle_lattice(D, c, w);
    if (Q < 0)
        return -1;
    return equilibrium_on(D, Q, c, w, kind, rho, u, feq);
}

/* Effective-viscosity factor A for a 1-D velocity u.
 *   entropic: eq. (entropic_bulk), with v = u / varsigma,
 *       A = 1 - (3/2) v^2 + (v^2 + 3 v^4 - 2 sqrt(v^2 + 1) + 2) / (2 v^2 + 2);
 *   polynomial (poly2 and product form): eq. (LBGK_bulk),
 *       A = 1 - (3/2) u^2 / varsigma^2. */
double oracle_bulk_A(int kind, double u)
{
    double v2 = (u * u) / CS2;
    if (kind == ORACLE_EQ_ENTROPIC)
        return 1.0 - 1.5 * v2 + (v2 + 3.0 * v2 * v2 - 2.0 * sqrt(v2 + 1.0) + 2.0) / (2.0 * v2 + 2.0);
    return 1.0 - 1.5 * v2;
}

/* Relaxation frequency beta at one node (the collision uses 2 beta).
 * nu = varsigma^2 (tau - 1/2); eq. (relaxation_frequency) without correction,
 * eq. (redefined_relaxation rate) with it, where the node's A is combined from
 * the per-axis A(u_alpha) by corr_mode. */
double oracle_beta(int D, int kind, int corr_mode, double tau, const double *u)
{
    double nu = CS2 * (tau - 0.5);
    if (corr_mode == ORACLE_CORR_OFF)
        return 1.0 / (2.0 * nu / CS2 + 1.0);
    double A = (corr_mode == ORACLE_CORR_MIN) ? INFINITY : 1.0;
    for (int a = 0; a < D; a++) {
        double Aa = oracle_bulk_A(kind, u[a]);
        if (corr_mode == ORACLE_CORR_MIN)
            A = (Aa < A) ? Aa : A;
        else
            A *= Aa;
    }
    return 1.0 / (2.0 * nu / (A * CS2) + 1.0);
}

/* Zeroth and first moments of one node's populations (Sec. "Discrete entropic
 * equilibrium construction": rho = sum f_i, rho u = sum c_i f_i). */
static void node_moments(int D, int Q, const int *c, const double *f, double *rho, double *u)
{
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; i++) {
        r += f[i];
        for (int a = 0; a < D; a++)
            j[a] += c[3 * i + a] * f[i];
    }
    *rho = r;
    for (int a = 0; a < D; a++)
        u[a] = j[a] / r;
}

/* One collision at a node: f <- f + 2 beta (f^eq - f).  Returns 1 if the node's
 * moments are outside the equilibrium's domain. */
static int node_collide(int D, int Q, const int *c, const double *w, int kind, int corr_mode,
                        double tau, double *f)
{
    double rho, u[3] = {0.0, 0.0, 0.0}, feq[27];
    node_moments(D, Q, c, f, &rho, u);
    int bad = equilibrium_on(D, Q, c, w, kind, rho, u, feq);
    double beta = oracle_beta(D, kind, corr_mode, tau, u);
    for (int i = 0; i < Q; i++)
        f[i] = f[i] + 2.0 * beta * (feq[i] - f[i]);
    return bad;
}

static long wrap(long x, long n)
{
    long r = x % n;
    return r < 0 ? r + n : r;
}

/* Run `steps` LBGK steps on a periodic nx * ny * nz grid (ny = nz = 1 for D = 1,
 * nz = 1 for D = 2) from f = f^eq(rho0, u0).
 * rho0: N values; u0: D planes of N values; x fastest.
 * Outputs rho (N) and u (D * N) after the last step, computed from the
 * pre-collision populations; f_out (Q * N, oracle ordering) if not NULL.
 * Returns the number of (node, step) pairs whose moments left the
 * equilibrium's domain (0 for a clean run), or -1 for bad arguments or memory. */
long oracle_run(int D, long nx, long ny, long nz, double tau, int kind, int corr_mode,
                const double *rho0, const double *u0, long steps,
                double *rho, double *u, double *f_out)
{
    int c[27 * 3];
    double w[27];
    int Q = oracle_lattice(D, c, w);
    if (Q < 0 || nx < 1 || ny < 1 || nz < 1 || steps < 0)
        return -1;
    if ((D < 3 && nz != 1) || (D < 2 && ny != 1))
        return -1;
    long N = nx * ny * nz;
    double *f = (double *)malloc(sizeof(double) * Q * N);
    double *g = (double *)malloc(sizeof(double) * Q * N);
    if (!f || !g) {
        free(f);
        free(g);
        return -1;
    }
    long bad = 0;

    for (long n = 0; n < N; n++) {
        double un[3] = {0.0, 0.0, 0.0}, feq[27];
        for (int a = 0; a < D; a++)
            un[a] = u0[a * N + n];
        bad += equilibrium_on(D, Q, c, w, kind, rho0[n], un, feq);
        for (int i = 0; i < Q; i++)
            f[i * N + n] = feq[i];
    }

    for (long t = 0; t < steps; t++) {
        long bad_step = 0;
#pragma omp parallel for reduction(+ : bad_step) schedule(static)
        for (long n = 0; n < N; n++) {
            long x = n % nx, y = (n / nx) % ny, z = n / (nx * ny);
            double fn[27];
            for (int i = 0; i < Q; i++)
                fn[i] = f[i * N + n];
            bad_step += node_collide(D, Q, c, w, kind, corr_mode, tau, fn);
            /* streaming: the post-collision value moves to r + c_i */
            for (int i = 0; i < Q; i++) {
                long xd = wrap(x + c[3 * i + 0], nx);
                long yd = wrap(y + c[3 * i + 1], ny);
                long zd = wrap(z + c[3 * i + 2], nz);
                g[i * N + xd + nx * (yd + ny * zd)] = fn[i];
            }
        }
        bad += bad_step;
        double *tmp = f;
        f = g;
        g = tmp;
    }

    for (long n = 0; n < N; n++) {
        double fn[27], r, un[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < Q; i++)
            fn[i] = f[i * N + n];
        node_moments(D, Q, c, fn, &r, un);
        if (rho)
            rho[n] = r;
        if (u)
            for (int a = 0; a < D; a++)
                u[a * N + n] = un[a];
    }
    if (f_out)
        memcpy(f_out, f, sizeof(double) * Q * N);
    free(f);
    free(g);
    return bad;
}

/* Sampled outputs of the same run for grids too large to step whole: the
 * moments at each sample node after `steps` steps.  A node's value after s
 * steps depends only on the initial state within distance s (Chebyshev), so
 * each sample is computed on its own box of side 2 s + 1 around it (periodic
 * images taken from the full initial field), stepped with open edges; the
 * corrupted edge region grows by one node per step and never reaches the
 * centre.  The box lies on the periodic extension of the grid, so it may be
 * larger than the grid itself.  Returns 0, or -1 for bad arguments or memory. */
long oracle_run_sample(int D, long nx, long ny, long nz, double tau, int kind, int corr_mode,
                       const double *rho0, const double *u0, long steps, long nsamples,
                       const long *sx, const long *sy, const long *sz,
                       double *rho_s, double *u_s)
{
    int c[27 * 3];
    double w[27];
    int Q = oracle_lattice(D, c, w);
    long ext[3] = {nx, ny, nz};
    if (Q < 0 || steps < 0 || nsamples < 0)
        return -1;
    if ((D < 3 && nz != 1) || (D < 2 && ny != 1))
        return -1;
    long L[3] = {1, 1, 1};
    for (int a = 0; a < D; a++)
        L[a] = 2 * steps + 1;
    if (nx < 1 || ny < 1 || nz < 1)
        return -1;
    long NB = L[0] * L[1] * L[2];
    long N = nx * ny * nz;
    double *f = (double *)malloc(sizeof(double) * Q * NB);
    double *g = (double *)malloc(sizeof(double) * Q * NB);
    if (!f || !g) {
        free(f);
        free(g);
        return -1;
    }
    for (long s = 0; s < nsamples; s++) {
        long centre[3] = {sx[s], D > 1 ? sy[s] : 0, D > 2 ? sz[s] : 0};
        for (long b = 0; b < NB; b++) {
            long loc[3] = {b % L[0], (b / L[0]) % L[1], b / (L[0] * L[1])};
            long gl[3];
            for (int a = 0; a < 3; a++)
                gl[a] = (a < D) ? wrap(centre[a] - steps + loc[a], ext[a]) : 0;
            long n = gl[0] + nx * (gl[1] + ny * gl[2]);
            double un[3] = {0.0, 0.0, 0.0}, feq[27];
            for (int a = 0; a < D; a++)
                un[a] = u0[a * N + n];
            equilibrium_on(D, Q, c, w, kind, rho0[n], un, feq);
            for (int i = 0; i < Q; i++)
                f[i * NB + b] = feq[i];
        }
        for (long t = 0; t < steps; t++) {
            for (long k = 0; k < Q * NB; k++)
                g[k] = 0.0;
#pragma omp parallel for schedule(static)
            for (long b = 0; b < NB; b++) {
                long loc[3] = {b % L[0], (b / L[0]) % L[1], b / (L[0] * L[1])};
                double fn[27];
                for (int i = 0; i < Q; i++)
                    fn[i] = f[i * NB + b];
                node_collide(D, Q, c, w, kind, corr_mode, tau, fn);
                for (int i = 0; i < Q; i++) {
                    long d[3];
                    int inside = 1;
                    for (int a = 0; a < 3; a++) {
                        d[a] = loc[a] + c[3 * i + a];
                        if (d[a] < 0 || d[a] >= L[a])
                            inside = 0;
                    }
                    if (inside)
                        g[i * NB + d[0] + L[0] * (d[1] + L[1] * d[2])] = fn[i];
                }
            }
            double *tmp = f;
            f = g;
            g = tmp;
        }
        long mid = steps + L[0] * ((D > 1 ? steps : 0) + L[1] * (D > 2 ? steps : 0));
        double fn[27], r, un[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < Q; i++)
            fn[i] = f[i * NB + mid];
        node_moments(D, Q, c, fn, &r, un);
        rho_s[s] = r;
        for (int a = 0; a < D; a++)
            u_s[a * nsamples + s] = un[a];
    }
    free(f);
    free(g);
    return 0;
}

/* Thread count of the node loops (OpenMP); returns the count in effect. */
int oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* Sec. "von Neumann spectral analysis: introduction" and the appendix
 * "Jacobian of entropic equilibrium": the Jacobian J_ij = d Omega_i / d f_j
 * of the collision operator Omega_i = 2 beta (f_i^eq - f_i), evaluated at the
 * equilibrium state f = f^eq(rho, u).
 *
 * At that state f^eq - f = 0, so the velocity dependence of beta under the
 * bulk correction contributes nothing: J = 2 beta(u) (d f^eq / d f - I).
 * d f^eq / d f follows from the chain rule through the moments,
 *     d rho / d f_j = 1,   d u_a / d f_j = (c_ja - u_a) / rho.
 * Entropic equilibrium, written as f_i^eq = w_i rho prod_a Lambda_a Gamma_ia
 * with Lambda_a = 2 - S_a, Gamma_ia = Z_a^{c_ia}, Z_a = (2 u_a + S_a) / (1 - u_a):
 *     d f_i^eq / d f_j = f_i^eq [ d ln rho + sum_a (d ln Lambda_a + d ln Gamma_ia) ],
 *     d S_a / d f_j = ((c_ja u_a / varsigma^2 + 1) / S_a - S_a) / rho,
 *     d ln Lambda_a / d f_j = -(d S_a / d f_j) / Lambda_a,
 *     d ln Gamma_ia / d f_j = c_ia [ (2 d u_a + d S_a) / (2 u_a + S_a) + d u_a / (1 - u_a) ].
 * (The printed derivative of Gamma is garbled; the last line is the
 * derivative of c_ia ln Z_a.)
 * Second-order polynomial equilibrium: its closed form differentiated in rho
 * and u.  Product form: f_i^eq = rho prod_a phi_{c_ia}(u_a) with
 * phi_0 = 1 - varsigma^2 - u^2 and phi_{+-1} = (+-u + varsigma^2 + u^2) / 2, so
 * d phi_0 / du = -2 u and d phi_{+-1} / du = (+-1 + 2 u) / 2.
 *
 * J is written row-major (J[i * Q + j]) in the oracle's population order.
 * Returns Q, or -1 for bad arguments. */
int oracle_jacobian(int D, int kind, int corr_mode, double tau, double rho, const double *u, double *J)
{
    int c[27 * 3];
    double w[27], feq[27];
    int Q = oracle_lattice(D, c, w);
    if (Q < 0 || !(rho > 0.0) || !(tau > 0.5))
        return -1;
    if (equilibrium_on(D, Q, c, w, kind, rho, u, feq) < 0)
        return -1;
    double two_beta = 2.0 * oracle_beta(D, kind, corr_mode, tau, u);

    for (int j = 0; j < Q; j++) {
        double du[3] = {0.0, 0.0, 0.0}; /* d u_a / d f_j */
        for (int a = 0; a < D; a++)
            du[a] = (c[3 * j + a] - u[a]) / rho;
        for (int i = 0; i < Q; i++) {
            double dfeq;
            if (kind == ORACLE_EQ_ENTROPIC) {
                double dlog = 1.0 / rho; /* d ln rho / d f_j */
                for (int a = 0; a < D; a++) {
                    double S = sqrt((u[a] * u[a]) / CS2 + 1.0);
                    double dS = ((c[3 * j + a] * u[a] / CS2 + 1.0) / S - S) / rho;
                    double Lambda = 2.0 - S;
                    dlog += -dS / Lambda;
                    dlog += c[3 * i + a] * ((2.0 * du[a] + dS) / (2.0 * u[a] + S) + du[a] / (1.0 - u[a]));
                }
                dfeq = feq[i] * dlog;
            } else if (kind == ORACLE_EQ_POLY2) {
                double cu = 0.0, usq = 0.0;
                for (int a = 0; a < D; a++) {
                    cu += c[3 * i + a] * u[a];
                    usq += u[a] * u[a];
                }
                double bracket = 1.0 + cu / CS2 + (cu * cu) / (2.0 * CS2 * CS2) - usq / (2.0 * CS2);
                dfeq = w[i] * bracket; /* d rho / d f_j = 1 */
                for (int a = 0; a < D; a++) {
                    double dbracket_du = c[3 * i + a] / CS2 + cu * c[3 * i + a] / (CS2 * CS2) - u[a] / CS2;
                    dfeq += w[i] * rho * dbracket_du * du[a];
                }
            } else {
                double phi[3], dphi[3];
                for (int a = 0; a < D; a++) {
                    int ca = c[3 * i + a];
                    if (ca == 0) {
                        phi[a] = 1.0 - CS2 - u[a] * u[a];
                        dphi[a] = -2.0 * u[a];
                    } else {
                        phi[a] = (ca * u[a] + CS2 + u[a] * u[a]) / 2.0;
                        dphi[a] = (ca + 2.0 * u[a]) / 2.0;
                    }
                }
                double prod = 1.0;
                for (int a = 0; a < D; a++)
                    prod *= phi[a];
                dfeq = prod; /* d rho / d f_j = 1 */
                for (int a = 0; a < D; a++) {
                    double others = 1.0;
                    for (int b = 0; b < D; b++)
                        if (b != a)
                            others *= phi[b];
                    dfeq += rho * others * dphi[a] * du[a];
                }
            }
            J[i * Q + j] = two_beta * (dfeq - (i == j ? 1.0 : 0.0));
        }
    }
    return Q;
}
