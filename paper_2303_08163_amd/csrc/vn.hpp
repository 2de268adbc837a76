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
// c x + s y for real c and complex s, as three-term fused sums per component
// (one multiplication and two fused multiply-adds each): the form in which
// rotations are applied.
__host__ __device__ __forceinline__ cplx crot(double c, cplx x, cplx s, cplx y) {
    return {fma(c, x.re, fma(s.re, y.re, -(s.im * y.im))), fma(c, x.im, fma(s.re, y.im, s.im * y.re))};
}
// w + conj(a) b and w - a b as two fused multiply-adds per component.
__host__ __device__ __forceinline__ cplx cmulc_add(cplx a, cplx b, cplx w) {
    return {fma(a.re, b.re, fma(a.im, b.im, w.re)), fma(a.re, b.im, fma(-a.im, b.re, w.im))};
}
__host__ __device__ __forceinline__ cplx cmul_sub(cplx a, cplx b, cplx w) {
    return {fma(-a.re, b.re, fma(a.im, b.im, w.re)), fma(-a.re, b.im, fma(-a.im, b.re, w.im))};
}
// Principal square root of z for O(1) entries: the modulus from the squared
// norm (no rescaling), one division, the sign cases selected (z = 0 gives 0).
__host__ __device__ __forceinline__ cplx csqrt_sq(cplx z) {
    const double r = sqrt(fma(z.re, z.re, z.im * z.im));
    const double t = sqrt(0.5 * (r + fabs(z.re)));
    const double h = 0.5 * z.im / (t > 0.0 ? t : 1.0);  // im / (2 t)
    const cplx pos = {t, h}, neg = {fabs(h), z.im >= 0.0 ? t : -t};
    const cplx w = z.re >= 0.0 ? pos : neg;
    return t > 0.0 ? w : cplx{0.0, 0.0};
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
    // E_ii = exp(-i c_i . k) = ex^(-c_x) ey^(-c_y) with ex = exp(i k_x),
    // ey = exp(i k_y): two sine-cosine pairs, products for the diagonal moves
    const cplx ex = {cos(k[0]), sin(k[0])};
    const cplx ey = DIM == 2 ? cplx{cos(k[1]), sin(k[1])} : cplx{1.0, 0.0};
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
        const cplx fx = cx < 0 ? ex : cplx{ex.re, -ex.im};  // ex^(-c_x) for c_x != 0
        const cplx fy = cy < 0 ? ey : cplx{ey.re, -ey.im};
        const cplx e = cx == 0 ? (cy == 0 ? cplx{1.0, 0.0} : fy) : (cy == 0 ? fx : cmul(fx, fy));
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

// 1 / sqrt(p) for p > 0 in the normal range: the hardware reciprocal square
// root estimate refined by two Newton-Raphson steps y <- y (3 - p y^2) / 2,
// each of which squares the relative error (the result is within a few ulp).
// p = 0 gives NaN; callers select another value then.
__host__ __device__ __forceinline__ double rsqrt_nr(double p) {
#if defined(__HIP_DEVICE_COMPILE__)
    double y = __builtin_amdgcn_rsq(p);
#else
    double y = (1.0 / sqrt(p)) * (1.0 + 3e-8);  // host stand-in for the estimate
#endif
    const double h = 0.5 * p;
    y = fma(y, fma(-h * y, y, 0.5), y);
    y = fma(y, fma(-h * y, y, 0.5), y);
    return y;
}

// Unitary Givens rotation G = [[c, s], [-conj(s), c]] (c real) with
// G (a, b)^T = (r, 0)^T; exactly the identity when b = 0.
//
// c = |a| / r and s = (a / |a|) conj(b) / r come from the squared norms with
// one reciprocal square root, q = 1 / sqrt(|a|^2 r^2): c = |a|^2 q and
// s = q a conj(b).  The cases are not branched on (branches here made the
// compiler hold much of the matrix twice):
// - b = 0 (or |b|^2 below 1e-162): c is set to 1 and s comes out 0 (q is
//   finite), so the rotation is exactly the identity;
// - |a|^2 < 1e-150: a is dropped, q = 1 / |b| and a + 1 stands for the unit
//   phase of a, so s = conj(b) / |b| and c = |a|^2 q ~ 0, each to a relative
//   1e-75.  Entries here are O(1) and a live b is above ulp times the
//   matrix scale (smaller ones are deflated to exact zeros), so neither is
//   above rounding, and otherwise |a|^2 r^2 >= 1e-300 stays normal.
__host__ __device__ __forceinline__ void givens(cplx a, cplx b, double &c, cplx &s) {
    const double na2 = fma(a.re, a.re, a.im * a.im), nb2 = fma(b.re, b.re, b.im * b.im);
    const bool drop_a = na2 < 1e-150;
    const double q = rsqrt_nr(drop_a ? fmax(nb2, 1e-300) : na2 * (na2 + nb2));
    const cplx ap = {a.re + (drop_a ? 1.0 : 0.0), a.im};
    c = nb2 == 0.0 ? 1.0 : na2 * q;
    s = cscale(q, cmul(ap, {b.re, -b.im}));
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
        // a column below 1e-130 needs no reflection: the QR iteration reads only
        // the Hessenberg part, so its entries below the subdiagonal count as
        // zeros (a perturbation of that size; exact when the column is zero)
        if (nrm2 <= 1e-260)
            return;
        const double alpha = sqrt(nrm2);
        // |x0| and the phase of x0 from one refined reciprocal square root (the
        // phase taken as 1 when |x0|^2 <= 1e-300, where v^H v below is then off
        // by a relative |x0| / alpha < 1e-20)
        const cplx x0 = A[k + 1][k];
        const double n0 = fma(x0.re, x0.re, x0.im * x0.im);
        const bool has_phase = n0 > 1e-300;
        const double r0 = rsqrt_nr(has_phase ? n0 : 1.0);
        const double ax0 = has_phase ? n0 * r0 : 0.0;
        const cplx ph = has_phase ? cscale(r0, x0) : cplx{1.0, 0.0};
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
                w = cmulc_add(v[i], A[i][j], w);
            });
            w = cscale(tau2, w);
            static_for<k + 1, N>([&](auto ii) {
                constexpr int i = decltype(ii)::value;
                A[i][j] = cmul_sub(v[i], w, A[i][j]);
            });
        });
        // right: A <- A H (all rows, columns k+1..N-1)
        static_for<0, N>([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            cplx w = {0.0, 0.0};
            static_for<k + 1, N>([&](auto jj) {
                constexpr int j = decltype(jj)::value;
                w = cmulc_add({A[i][j].re, -A[i][j].im}, v[j], w);  // w + A v
            });
            w = cscale(tau2, w);
            static_for<k + 1, N>([&](auto jj) {
                constexpr int j = decltype(jj)::value;
                A[i][j] = cmul_sub(w, {v[j].re, -v[j].im}, A[i][j]);
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
// (hi > M - 1 never happens: M - 1 is the wavefront's largest hi).  Rows
// below hi are deflated (zero subdiagonal), the rotations there are exact
// identities, so without the shift their values are left unchanged (a zero
// may change sign).
//
// R Q applies the column rotation k to rows 0..k+1 of columns k, k+1; those
// rows are final in R once the row rotation k+1 is done, and no later row
// rotation reads or writes them.  So column rotation k runs right after row
// rotation k+1: every entry sees the same operations in the same order as
// with all row rotations first, and only two rotations are live at a time
// (which keeps the matrix in registers).
template <int N, int M>
__host__ __device__ __forceinline__ void qr_step(cplx (&H)[N][N], cplx mu, int hi) {
    // the shift on rows 0..hi: f = 1 there subtracts mu exactly as a
    // subtraction rounds, f = 0 leaves the row's value as it is
    static_for<0, M>([&](auto kk) {
        constexpr int k = decltype(kk)::value;
        const double f = k <= hi ? 1.0 : 0.0;
        H[k][k] = {fma(-f, mu.re, H[k][k].re), fma(-f, mu.im, H[k][k].im)};
    });
    // columns k, k+1 times G_k^H: col k <- c x + conj(s) y ; col k+1 <- -s x + c y
    auto column_rotation = [&](auto kk, double c, cplx s) {
        constexpr int k = decltype(kk)::value;
        static_for<0, k + 1>([&](auto ii) {
            constexpr int i = decltype(ii)::value;
            const cplx x = H[i][k], y = H[i][k + 1];
            H[i][k] = crot(c, x, {s.re, -s.im}, y);
            H[i][k + 1] = crot(c, y, {-s.re, -s.im}, x);
        });
        // row k + 1: its column-k entry is the exact zero row rotation k left,
        // so the terms with it drop out (the same values; a zero may change sign)
        const cplx y = H[k + 1][k + 1];
        H[k + 1][k] = cmul({s.re, -s.im}, y);
        H[k + 1][k + 1] = cscale(c, y);
    };
    double c_prev = 1.0;
    cplx s_prev = {0.0, 0.0};
    static_for<0, M - 1>([&](auto kk) {
        constexpr int k = decltype(kk)::value;
        double c;
        cplx s;
        givens(H[k][k], H[k + 1][k], c, s);
        static_for<k, M>([&](auto jj) {
            constexpr int j = decltype(jj)::value;
            const cplx x = H[k][j], y = H[k + 1][j];
            // row k <- c x + s y ; row k+1 <- -conj(s) x + c y
            H[k][j] = crot(c, x, s, y);
            H[k + 1][j] = crot(c, y, {-s.re, s.im}, x);
        });
        H[k + 1][k] = {0.0, 0.0};
        if constexpr (k > 0)
            column_rotation(std::integral_constant<int, k - 1>{}, c_prev, s_prev);
        c_prev = c;
        s_prev = s;
    });
    column_rotation(std::integral_constant<int, M - 2>{}, c_prev, s_prev);
    static_for<0, M>([&](auto kk) {
        constexpr int k = decltype(kk)::value;
        const double f = k <= hi ? 1.0 : 0.0;
        H[k][k] = {fma(f, mu.re, H[k][k].re), fma(f, mu.im, H[k][k].im)};
    });
}

// Operation counts, used to report the solver's arithmetic rate: the FP64
// operations the code performs for one matrix's own work.  Additions,
// subtractions, multiplications, divisions, square roots, sines and cosines
// count 1, a fused multiply-add 2, the refined reciprocal square root 2 (as the
// square root and division it stands for); absolute values, maxima,
// comparisons, selects and negations count 0.  A QR step counts the matrix's
// own active block of m rows, not the wavefront's common one, and the shift's
// subtraction and return 1 per component each (written as fused multiply-adds
// with a factor 0 or 1).
//
// Building M (vn_matrix, without or with the correction's relaxation rate).
template <int DIM, int EQ, bool CORR>
__host__ __device__ constexpr double vn_build_flops() {
    constexpr double N = DIM == 1 ? 3.0 : 9.0;
    // per axis: the factors g_c(u_a) and their derivatives (entropic: S,
    // the three factors, u / S and three derivatives; product form: seven
    // for the factors, three derivatives)
    const double axis = EQ == kEqEntropic ? 16.0 : (EQ == kEqProduct ? 10.0 : 0.0);
    // per population: U_0 and U_a (product forms: products of factors; the
    // polynomial: c.u, U_0 and U_a from it), once: u^2, 1 - 1.5 u^2, 3 u_a
    const double per_i = EQ == kEqPoly2 ? (DIM - 1.0) + 5.0 + 5.0 * DIM : (DIM == 2 ? 3.0 : 0.0);
    const double once = EQ == kEqPoly2 ? 2.0 * DIM + 2.0 + DIM : 0.0;
    const double omega = !CORR ? 1.0 : (EQ == kEqEntropic ? 25.0 : 8.0);
    // sin and cos of each k_a; the four diagonal moves' phase products
    const double phases = 2.0 * DIM + (DIM == 2 ? 4.0 * 6.0 : 0.0);
    // c_ja - u_a; per entry P_ij (one fused multiply-add per axis), omega P_ij,
    // times E_ii (2); the diagonal's 1 - omega and its addition
    const double entries = 3.0 * DIM + N * N * (2.0 * DIM + 3.0) + 1.0 + N;
    return DIM * axis + N * per_i + once + omega + phases + entries;
}
// The Householder reduction (a reflector of length m = N - 1 .. 2: its norm
// 4 m, alpha, |x0| and phase 9, v 4, tau 3, the left update m (16 m + 2), the
// right update N (16 m + 2), the new subdiagonal 2), the deflation scan before
// the first step (5 per row), the norm of the Hessenberg part (one addition per
// entry, times 1e-2) and the radius (|lambda|^2 of each eigenvalue, one square
// root).
template <int N>
__host__ __device__ constexpr double vn_reduce_flops() {
    double h = 0.0;
    for (int m = 2; m <= N - 1; ++m)
        h += 16.0 * m * m + (6.0 + 16.0 * N) * m + 2.0 * N + 18.0;
    const double deflation = 5.0 * (N - 1);
    const double norm = N * (N + 1) / 2 + (N - 1) + 1.0;
    const double radius = 3.0 * N + 1.0;
    return h + deflation + norm + radius;
}
// One QR step on an active block of m rows.  Per rotation: forming it (20)
// and applying it to rows k, k + 1 of columns k..m-1 (10 for column k, whose
// lower entry is set to zero, 20 for each other) and to rows 0..k+1 of columns
// k, k + 1 (20 each, 8 for row k + 1, whose column-k entry is zero): 20 m + 38.
// Per step: the deflation scan (5 per row below the first), the shift (52: the
// trailing 2 x 2's eigenvalue nearer its last diagonal entry and the
// exceptional shift, both formed) and its subtraction and return on the
// block's rows (4 m).
__host__ __device__ constexpr double vn_step_flops(int m) {
    return (m - 1) * (20.0 * m + 43.0) + 4.0 * m + 52.0;
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
// thread of the group is done; a finished thread's steps leave its values
// unchanged.
//
// The group's M never grows: a zero subdiagonal entry stays exactly zero
// (its rotation is the identity) and a thread that gives up reports hi = 0
// from then on.  So the iteration is a sequence of loops, one per block size
// from N down to 2, each running while M has its size; the deflation scan and
// the shift then look at the rows of that block only (the rows below are
// deflated in every thread that is still iterating).
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
    // deflate negligible subdiagonal entries of rows 1..M-1 (relative to their
    // diagonal neighbours, or to the matrix norm when those are tiny); returns
    // hi = the lowest unreduced row, 0 once the iteration limit is reached
    auto deflate = [&](auto mm) {
        constexpr int M = decltype(mm)::value;
        int h = 0;
        static_for<1, M>([&](auto kk) {
            constexpr int k = decltype(kk)::value;
            const double scale = fmax(cabs1(H[k][k]) + cabs1(H[k - 1][k - 1]), norm);
            // kept entries are nonzero (and a NaN is kept), so one comparison
            // decides both
            const bool keep = !(cabs1(H[k][k - 1]) <= kUlp * scale);
            H[k][k - 1] = keep ? H[k][k - 1] : cplx{0.0, 0.0};
            h = keep ? k : h;
        });
        if (h > 0 && steps >= 30 * N) {
            failed = true;
            h = 0;  // give up: stop stepping this matrix
        }
        return h;
    };
    int hi = deflate(std::integral_constant<int, N>{});
    int wave_hi = group_max(hi);
    static_for<0, N - 1>([&](auto dd) {
        constexpr int M = N - decltype(dd)::value;  // N, N - 1, ..., 2
        while (wave_hi + 1 == M) {
            // shift from the trailing 2 x 2 of this thread's active block,
            // [[a, b], [c, d]] at rows hi-1, hi (zero when hi = 0, where the
            // shift is not used); computed without branches, cases selected
            cplx a = {0.0, 0.0}, b = a, c = a, d = a;
            double e1 = 0.0;  // |H[hi-1][hi-2]| (1-norm; 0 if hi = 1)
            static_for<1, M>([&](auto kk) {
                constexpr int k = decltype(kk)::value;
                if (k == hi) {
                    a = H[k - 1][k - 1];
                    b = H[k - 1][k];
                    c = H[k][k - 1];
                    d = H[k][k];
                    if constexpr (k >= 2)
                        e1 = cabs1(H[k - 1][k - 2]);
                }
            });
            const bool active = hi > 0;
            const bool fresh = hi != last_hi;
            last_hi = active && fresh ? hi : last_hi;
            since_deflation = active && fresh ? 0 : since_deflation;
            // Wilkinson: the eigenvalue of the 2 x 2 closer to d, d - b c / den,
            // with den = half +- disc (disc^2 = half^2 + b c) the one of larger
            // size (for stability)
            const cplx half = cscale(0.5, csub(a, d));
            const cplx bc = cmul(b, c);
            const cplx disc = csqrt_sq(cadd(cmul(half, half), bc));
            const cplx m1 = cadd(half, disc), m2 = csub(half, disc);
            const cplx den = cabs1(m1) >= cabs1(m2) ? m1 : m2;
            const double den2 = fma(den.re, den.re, den.im * den.im);
            const double inv = 1.0 / (den2 > 0.0 ? den2 : 1.0);
            const cplx wil = csub(d, cscale(inv, cmulc({den.re, den.im}, bc)));
            const cplx wilk = den2 > 0.0 ? wil : d;
            // exceptional shift after 10 and 20 steps without deflation
            const bool exceptional = since_deflation == 10 || since_deflation == 20;
            const cplx exc = {d.re + 0.75 * (cabs1(c) + e1), d.im};
            const cplx mu_a = exceptional ? exc : wilk;
            const cplx mu = active ? mu_a : cplx{0.0, 0.0};
            steps += active ? 1 : 0;
            since_deflation += active ? 1 : 0;
            if (work)
                *work += active ? vn_step_flops(hi + 1) : 0.0;
            // one QR step on the leading M x M block, the same size for the group
            qr_step<N, M>(H, mu, hi);
            hi = deflate(std::integral_constant<int, M>{});
            wave_hi = group_max(hi);
        }
    });
    return failed ? -1 : steps;
}

}  // namespace lbm
