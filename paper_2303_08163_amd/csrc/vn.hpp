// vn.hpp -- von Neumann amplification matrices and their eigenvalues, one
// matrix per thread (Sec. "Linear stability analysis" of arXiv:2303.08163).
//
// A plane-wave perturbation of the uniform state (rho = 1, u) evolves by
// eq. (PerturbedDiscreteLBE); the amplification matrix is M = E (I + J)
// (eq. VN_eigen) with E_ii = exp(-i c_i . k) and J the collision Jacobian.
// At an equilibrium state f^eq - f = 0, so the velocity dependence of beta
// under the bulk correction drops out of J and
//     I + J = (1 - omega) I + omega P,   P = d f^eq / d f,   omega = 2 beta.
// Every equilibrium here is rho times a function of u, and the moments give
// d rho / d f_j = 1, d u_a / d f_j = (c_ja - u_a) / rho, so P has rank D + 1:
//     P_ij = U_i0 + sum_a U_ia (c_ja - u_a),
//     U_i0 = f_i^eq / rho,   U_ia = d (f_i^eq / rho) / d u_a.
// For the product-form equilibria (entropic and product form) f_i^eq / rho is
// prod_a g_{c_ia}(u_a), so U_ia = g'_{c_ia}(u_a) prod_{b != a} g_{c_ib}(u_b):
//     entropic:     g'_0 = -2 u / S,  g'_{+-1} = u / S +- 1/2   (S = sqrt(1 + 3 u^2));
//     product form: g'_0 = -2 u,      g'_{+-1} = u +- 1/2.
// The second-order polynomial equilibrium is differentiated directly.
//
// Eigenvalues: complex Householder reduction to upper Hessenberg form, then
// shifted QR steps (Wilkinson shift from the trailing 2 x 2 of the lowest
// unreduced block, exceptional shifts after 10 and 20 steps without
// deflation) until every subdiagonal entry is negligible.  All loops run
// over compile-time index ranges so the matrix stays in registers; a QR step
// sweeps the leading block that still holds unconverged eigenvalues of any
// thread of the wavefront (rotations against a zero subdiagonal are exact
// identities, so deflated blocks stay decoupled).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "node.hpp"

namespace lbm {

// Compile-time loop: f(std::integral_constant<int, i>) for i in [B, E).  Used
// where loop bounds depend on an outer index, which the unroller does not
// expand, so that every matrix index is a constant and the matrix stays in
// registers.
template <int B, int E, typename F>
__host__ __device__ __forceinline__ void static_for(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

struct cplx {
    double re, im;
};
__host__ __device__ __forceinline__ cplx cmul(cplx a, cplx b) {
    return {fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re)};
}
__host__ __device__ __forceinline__ cplx cmulc(cplx a, cplx b) {  // conj(a) * b
    return {fma(a.re, b.re, a.im * b.im), fma(a.re, b.im, -a.im * b.re)};
}
__host__ __device__ __forceinline__ cplx cadd(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
__host__ __device__ __forceinline__ cplx csub(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
__host__ __device__ __forceinline__ cplx cscale(double s, cplx a) { return {s * a.re, s * a.im}; }
__host__ __device__ __forceinline__ double cabs1(cplx a) { return fabs(a.re) + fabs(a.im); }
__host__ __device__ __forceinline__ double cabs(cplx a) { return hypot(a.re, a.im); }
__host__ __device__ __forceinline__ cplx csqrt_(cplx a) {
    // principal square root, written to avoid cancellation
    const double r = cabs(a);
    if (r == 0.0)
        return {0.0, 0.0};
    const double t = sqrt(0.5 * (r + fabs(a.re)));
    if (a.re >= 0.0)
        return {t, a.im / (2.0 * t)};
    return {fabs(a.im) / (2.0 * t), a.im >= 0.0 ? t : -t};
}
__host__ __device__ __forceinline__ cplx cdiv(cplx a, cplx b) {
    const double d = fma(b.re, b.re, b.im * b.im);
    return {fma(a.re, b.re, a.im * b.im) / d, fma(a.im, b.re, -a.re * b.im) / d};
}

// Relaxation omega = 2 beta at velocity u (lattice units, 2 beta = 1 / tau
// without the correction).
template <int DIM, int EQ, bool CORR>
__host__ __device__ __forceinline__ double vn_omega(double tau, const double (&u)[2]) {
    if (!CORR)
        return 1.0 / tau;
    double umax = fabs(u[0]);
    if (DIM == 2)
        umax = fmax(umax, fabs(u[1]));
    if (EQ == kEqEntropic)
        return corrected_omega(umax, sqrt(fma(3.0 * umax, umax, 1.0)), 2.0 * tau - 1.0);
    return corrected_omega_poly(umax, 2.0 * tau - 1.0);
}

// M = E ((1 - omega) I + omega P) for D1Q3 (DIM = 1, N = 3) or D2Q9
// (DIM = 2, N = 9); population i = cx + 3 cy with c = index - 1.
template <int DIM, int EQ, bool CORR>
__host__ __device__ __forceinline__ void vn_matrix(double tau, const double (&u)[2], const double (&k)[2],
                                                   cplx (&M)[DIM == 1 ? 3 : 9][DIM == 1 ? 3 : 9]) {
    constexpr int N = DIM == 1 ? 3 : 9;
    double g[2][3], dg[2][3];
    double usq = 0.0;
    for (int a = 0; a < DIM; ++a) {
        usq = fma(u[a], u[a], usq);
        if (EQ == kEqEntropic) {
            double S;
            axis_factors(u[a], g[a], S);
            const double uS = u[a] / S;
            dg[a][0] = uS - 0.5;
            dg[a][1] = -2.0 * uS;
            dg[a][2] = uS + 0.5;
        } else if (EQ == kEqProduct) {
            product_factors(u[a], g[a]);
            dg[a][0] = u[a] - 0.5;
            dg[a][1] = -2.0 * u[a];
            dg[a][2] = u[a] + 0.5;
        }
    }
    const double omega = vn_omega<DIM, EQ, CORR>(tau, u);
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const int cx = i % 3 - 1, cy = DIM == 2 ? i / 3 - 1 : 0;
        double U0, Ux, Uy = 0.0;
        if (EQ == kEqPoly2) {
            const double w = DIM == 1 ? w1(i) : w1(i % 3) * w1(i / 3);
            const double cu = cx * u[0] + (DIM == 2 ? cy * u[1] : 0.0);
            U0 = w * fma(cu, fma(4.5, cu, 3.0), fma(-1.5, usq, 1.0));
            Ux = w * (fma(9.0 * cu, cx, 3.0 * cx) - 3.0 * u[0]);
            if (DIM == 2)
                Uy = w * (fma(9.0 * cu, cy, 3.0 * cy) - 3.0 * u[1]);
        } else {
            const double gx = g[0][cx + 1], gy = DIM == 2 ? g[1][cy + 1] : 1.0;
            U0 = gx * gy;
            Ux = dg[0][cx + 1] * gy;
            if (DIM == 2)
                Uy = gx * dg[1][cy + 1];
        }
        // E_ii = exp(-i c_i . k)
        const double phase = -(cx * k[0] + (DIM == 2 ? cy * k[1] : 0.0));
        const cplx e = {cos(phase), sin(phase)};
#pragma unroll
        for (int j = 0; j < N; ++j) {
            const int jx = j % 3 - 1, jy = DIM == 2 ? j / 3 - 1 : 0;
            double p = fma(Ux, jx - u[0], U0);
            if (DIM == 2)
                p = fma(Uy, jy - u[1], p);
            const double a = omega * p + (i == j ? 1.0 - omega : 0.0);
            M[i][j] = cscale(a, e);
        }
    }
}

// Unitary Givens rotation G = [[c, s], [-conj(s), c]] (c real) with
// G (a, b)^T = (r, 0)^T; exactly the identity when b = 0.
//
// The rotations form the serial chain of a QR step, so they are computed from
// the squared norms with one square root and one division in sequence:
// q = 1 / sqrt(|a|^2 r^2) gives c = |a| / r = |a|^2 q and |s| scale 1 / (|a| r)
// = q.  Entries here are O(1) and deflation zeroes any below ulp times its
// scale, so the products neither overflow nor underflow; should they reach
// the underflow range anyway, the rescaling form below runs.
__host__ __device__ __forceinline__ void givens(cplx a, cplx b, double &c, cplx &s) {
    if (b.re == 0.0 && b.im == 0.0) {
        c = 1.0;
        s = {0.0, 0.0};
        return;
    }
    const double na2 = fma(a.re, a.re, a.im * a.im), nb2 = fma(b.re, b.re, b.im * b.im);
    const double r2 = na2 + nb2;
    if (na2 == 0.0 && r2 > 1e-300) {
        c = 0.0;
        s = cscale(1.0 / sqrt(r2), {b.re, -b.im});  // conj(b) / |b|
        return;
    }
    const double p = na2 * r2;
    if (p > 1e-300) {
        const double q = 1.0 / sqrt(p);
        c = na2 * q;
        // s = (a / |a|) conj(b) / r = a conj(b) q
        s = cscale(q, cmul(a, {b.re, -b.im}));
        return;
    }
    const double na = cabs(a), nb = cabs(b);
    if (na == 0.0) {
        c = 0.0;
        s = cscale(1.0 / nb, {b.re, -b.im});  // conj(b) / |b|
        return;
    }
    const double r = hypot(na, nb);
    c = na / r;
    // s = (a / |a|) conj(b) / r
    const cplx ph = cscale(1.0 / na, a);
    s = cscale(1.0 / r, cmul(ph, {b.re, -b.im}));
}

// Reduce A to upper Hessenberg form by Householder reflections (similarity).
template <int N>
__host__ __device__ __forceinline__ void hessenberg(cplx (&A)[N][N]) {
    static_for<0, N - 2>([&](auto kk) {
        constexpr int k = decltype(kk)::value;
        // reflector for x = A[k+1..N-1][k]: v = x + e^{i arg x0} |x| e_1
        double nrm2 = 0.0;
        static_for<k + 1, N>([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            nrm2 = fma(A[i][k].re, A[i][k].re, fma(A[i][k].im, A[i][k].im, nrm2));
        });
        const double alpha = sqrt(nrm2);
        if (alpha == 0.0)
            return;
        const cplx x0 = A[k + 1][k];
        const double ax0 = cabs(x0);
        const cplx ph = ax0 > 0.0 ? cscale(1.0 / ax0, x0) : cplx{1.0, 0.0};
        cplx v[N];
        v[k + 1] = cadd(x0, cscale(alpha, ph));
        static_for<k + 2, N>([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            v[i] = A[i][k];
        });
        // H = I - 2 v v^H / (v^H v);  v^H v = 2 alpha (alpha + |x0|)
        const double tau2 = 1.0 / (alpha * (alpha + ax0));
        // left: A <- H A (rows k+1..N-1, columns k+1..N-1; column k is set below)
        static_for<k + 1, N>([&](auto jj) {
            constexpr int j = decltype(jj)::value;
            cplx w = {0.0, 0.0};
            static_for<k + 1, N>([&](auto ii) {
                constexpr int i = decltype(ii)::value;
                w = cadd(w, cmulc(v[i], A[i][j]));
            });
            w = cscale(tau2, w);
            static_for<k + 1, N>([&](auto ii) {
                constexpr int i = decltype(ii)::value;
                A[i][j] = csub(A[i][j], cmul(v[i], w));
            });
        });
        // right: A <- A H (all rows, columns k+1..N-1)
        static_for<0, N>([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            cplx w = {0.0, 0.0};
            static_for<k + 1, N>([&](auto jj) {
                constexpr int j = decltype(jj)::value;
                w = cadd(w, cmul(A[i][j], v[j]));
            });
            w = cscale(tau2, w);
            static_for<k + 1, N>([&](auto jj) {
                constexpr int j = decltype(jj)::value;
                A[i][j] = csub(A[i][j], cmul(w, {v[j].re, -v[j].im}));
            });
        });
        // column k below the subdiagonal is annihilated: H x = -e^{i arg x0} alpha e_1
        A[k + 1][k] = cscale(-alpha, ph);
        static_for<k + 2, N>([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            A[i][k] = {0.0, 0.0};
        });
    });
}

// One explicit shifted QR step on the leading M x M block of H:
// H - mu I = Q R, H <- R Q + mu I, with the shift applied to rows 0..hi only
// (hi >= M - 1 never happens: M - 1 is the wavefront's largest hi).  Rows
// below hi are deflated (zero subdiagonal), the rotations there are exact
// identities, so without the shift they are left bit-for-bit unchanged.
template <int N, int M>
__host__ __device__ __forceinline__ void qr_step(cplx (&H)[N][N], cplx mu, int hi) {
    static_for<0, M>([&](auto kk) {
        constexpr int k = decltype(kk)::value;
        if (k <= hi)
            H[k][k] = csub(H[k][k], mu);
    });
    double cs[M - 1];
    cplx sn[M - 1];
    static_for<0, M - 1>([&](auto kk) {
        constexpr int k = decltype(kk)::value;
        givens(H[k][k], H[k + 1][k], cs[k], sn[k]);
        static_for<k, M>([&](auto jj) {
            constexpr int j = decltype(jj)::value;
            const cplx x = H[k][j], y = H[k + 1][j];
            // row k <- c x + s y ; row k+1 <- -conj(s) x + c y
            H[k][j] = cadd(cscale(cs[k], x), cmul(sn[k], y));
            H[k + 1][j] = csub(cscale(cs[k], y), cmulc(sn[k], x));
        });
        H[k + 1][k] = {0.0, 0.0};
    });
    static_for<0, M - 1>([&](auto kk) {
        constexpr int k = decltype(kk)::value;
        static_for<0, k + 2>([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            const cplx x = H[i][k], y = H[i][k + 1];
            // columns k, k+1 times G^H: col k <- c x + conj(s) y ; col k+1 <- -s x + c y
            H[i][k] = cadd(cscale(cs[k], x), cmulc(sn[k], y));
            H[i][k + 1] = csub(cscale(cs[k], y), cmul(sn[k], x));
        });
    });
    static_for<0, M>([&](auto kk) {
        constexpr int k = decltype(kk)::value;
        if (k <= hi)
            H[k][k] = cadd(H[k][k], mu);
    });
}

// FP64 operations (a fused multiply-add counts 2; divisions, square roots and
// transcendentals 1) of the solver as written: building M, the Householder
// reduction and the norm (fixed), and one QR step on an active block of M
// rows (its rotations, the shift on M rows, the deflation scan and the shift
// choice).  Used to report the arithmetic rate; they count each matrix's own
// active block, not the wavefront's common one.
template <int N>
__host__ __device__ constexpr double vn_fixed_flops() {
    double h = 0.0;
    for (int m = 2; m <= N - 1; ++m)
        h += 16.0 * m * m + (6.0 + 16.0 * N) * m + 2.0 * N + 14.0;
    const double build = 9.0 * N * N + 20.0 * N + 40.0;
    const double norm = 3.0 * (N * (N + 1) / 2 + N - 1) + 4.0 * N;
    return h + build + norm;
}
__host__ __device__ constexpr double vn_step_flops(int M) {
    // per rotation: applying it to two rows and two columns (20 M) and
    // forming it from squared norms (19) with the rest of its bookkeeping (46)
    return (M - 1) * (20.0 * M + 65.0) + 4.0 * M + 150.0;
}

// Eigenvalues of an upper Hessenberg matrix (overwritten; the diagonal holds
// them on return).  Returns the number of QR steps taken, or -1 if the
// iteration limit (30 N steps) was reached first.
//
// For eigenvalues only, once the rows below hi have deflated the leading
// (hi + 1) x (hi + 1) block carries every remaining eigenvalue, so a step
// sweeps only the leading M x M block.  group_max(v) returns the largest v
// over the threads that execute in lockstep (a wavefront on the GPU, the
// thread itself on the host); M is taken from it so that every thread of a
// wavefront runs the same compile-time block size.  Every thread must call
// this function (none may have left early), and the loop runs until every
// thread of the group is done; a finished thread's steps are exact no-ops.
template <int N, typename GroupMax>
__host__ __device__ __forceinline__ int hessenberg_eigenvalues(cplx (&H)[N][N], GroupMax group_max,
                                                               double *work = nullptr) {
    constexpr double kUlp = 2.220446049250313e-16;
    // scale below which a subdiagonal entry is negligible in any case:
    // ulp times 1e-2 times the largest |entry| (1-norm of the complex value)
    double norm = 0.0;
    static_for<0, N>([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        static_for<(i > 0 ? i - 1 : 0), N>([&](auto jj) {
            constexpr int j = decltype(jj)::value;
            norm = fmax(norm, cabs1(H[i][j]));
        });
    });
    norm *= 1e-2;
    int steps = 0, since_deflation = 0, last_hi = N;
    bool failed = false;
    for (;;) {
        // deflate negligible subdiagonal entries (relative to their diagonal
        // neighbours, or to the matrix norm when those are tiny); hi = lowest
        // unreduced row
        int hi = 0;
        static_for<1, N>([&](auto kk) {
            constexpr int k = decltype(kk)::value;
            const double scale = fmax(cabs1(H[k][k]) + cabs1(H[k - 1][k - 1]), norm);
            if (cabs1(H[k][k - 1]) <= kUlp * scale)
                H[k][k - 1] = {0.0, 0.0};
            if (H[k][k - 1].re != 0.0 || H[k][k - 1].im != 0.0)
                hi = k;
        });
        if (hi > 0 && steps >= 30 * N) {
            failed = true;
            hi = 0;  // give up: stop stepping this matrix
        }
        const int wave_hi = group_max(hi);
        if (wave_hi == 0)
            return failed ? -1 : steps;
        cplx mu = {0.0, 0.0};
        if (hi > 0) {
            if (hi != last_hi) {
                last_hi = hi;
                since_deflation = 0;
            }
            // trailing 2 x 2 of the active block: [[a, b], [c, d]] at rows hi-1, hi
            cplx a = {0.0, 0.0}, b = a, c = a, d = a, e = a;  // e = H[hi-1][hi-2] (0 if hi = 1)
            static_for<1, N>([&](auto kk) {
                constexpr int k = decltype(kk)::value;
                if (k == hi) {
                    a = H[k - 1][k - 1];
                    b = H[k - 1][k];
                    c = H[k][k - 1];
                    d = H[k][k];
                    if constexpr (k >= 2)
                        e = H[k - 1][k - 2];
                }
            });
            if (since_deflation == 10 || since_deflation == 20) {
                // exceptional shift
                const double t = cabs1(c) + cabs1(e);
                mu = {d.re + 0.75 * t, d.im};
            } else {
                // Wilkinson: eigenvalue of the 2 x 2 closer to d
                const cplx half = cscale(0.5, csub(a, d));
                const cplx disc = csqrt_(cadd(cmul(half, half), cmul(b, c)));
                const cplx m1 = cadd(half, disc), m2 = csub(half, disc);
                const cplx den = cabs1(m1) >= cabs1(m2) ? m1 : m2;  // larger root for stability
                mu = (den.re == 0.0 && den.im == 0.0) ? d : csub(d, cdiv(cmul(b, c), den));
            }
            ++steps;
            ++since_deflation;
            if (work)
                *work += vn_step_flops(hi + 1);
        }
        // one QR step on the leading (wave_hi + 1) block, the same size for the group
        static_for<2, N + 1>([&](auto mm) {
            constexpr int M = decltype(mm)::value;
            if (wave_hi + 1 == M)
                qr_step<N, M>(H, mu, hi);
        });
    }
}

}  // namespace lbm
