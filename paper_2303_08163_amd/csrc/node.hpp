// node.hpp -- per-node arithmetic of one LBGK step with the entropic
// equilibrium, shared by every kernel of the library so that a node's result
// is bitwise the same whichever kernel (single domain, batched, pool) runs it.
//
// Method (arXiv:2303.08163):
//   Sec. "Basic concepts": f_i <- f_i + 2 beta (f_i^eq - f_i), with
//     rho = sum_i f_i and rho u = sum_i c_i f_i; 2 beta = 1 / tau.
//   Sec. "Discrete entropic equilibrium construction", eq.
//     (Entropic_isothermal_EDF).  With S_a = sqrt(1 + 3 u_a^2) the multipliers
//     Z_a = (2 u_a + S_a) / (1 - u_a) and X^{-1} = rho prod_a (2 - S_a) give
//     f_i^eq = rho prod_a g_{c_ia}(u_a), where
//       g_0 = 2 (2 - S) / 3,  g_{+1} = (2 S - 1 + 3 u) / 6,  g_{-1} = (2 S - 1 - 3 u) / 6
//     because, with S^2 = 1 + 3 u^2, (2 - S)(2 u + S) = (1 - u)(2 S - 1 + 3 u) and
//     (2 - S)(1 - u) = (2 u + S)(2 S - 1 - 3 u) hold identically.  This needs
//     one square root per axis and no power, exponential or division.  The
//     factors are formed as h +- u/2 and 1 - 2 h with h = (2 S - 1) / 6, so
//     that g_{+1} - g_{-1} = u and g_{-1} + g_0 + g_{+1} = 1 hold up to
//     value-dependent rounding: multiplying every factor by a rounded constant
//     (1/6, 2/3) would remove the same fraction of mass and momentum at every
//     node and step, a bias that adds up over long runs.
//   Sec. "Correction of leading-order bulk viscosity error", eq.
//     (redefined_relaxation rate) with A from eq. (entropic_bulk):
//     2 beta = 2 A / (A + 2 tau - 1).  A node uses A = min_a A(u_a); A is even
//     and decreasing in |u| on [0, 1), so that is A at u_max = max_a |u_a|, i.e.
//     at S_max = max_a S_a.  Written without cancellation
//     (v^2 = 3 u_max^2, v^2 + 2 - 2 S = (S - 1)^2 = v^4 / (S + 1)^2):
//       A = [2 S^2 (S+1)^2 (1 - 3 v^2 / 2) + v^4 (3 (S+1)^2 + 1)] / [2 S^2 (S+1)^2],
//     so 2 beta = 2 P / (P + (2 tau - 1) Qd) with A = P / Qd: one division.
//
// Storage: DEV = false holds f_i in double.  DEV = true holds deviations
// f_i - w_i rho0 in float; the moments use sum w_i = 1 and sum w_i c_i = 0 so
// that rho = rho0 + sum_i (f_i - w_i rho0) and rho u = sum_i c_i (f_i - w_i rho0).
// All arithmetic is double.  The library is compiled with FMA contraction off;
// the fused multiply-adds below are written out.
//
// Population index: i = (c_x + 1) + 3 (c_y + 1) + 9 (c_z + 1) (D1Q3: i = c_x + 1).
#pragma once

#include <hip/hip_runtime.h>

namespace lbm {

// Storage and arithmetic of a domain (the values of lbm_config.dtype):
//   kF64:        double storage, double arithmetic;
//   kDevF64:     float deviations f_i - w_i rho0, all arithmetic in double;
//   kDevMixed:   float deviations; moments, square roots and the per-axis
//                factor deviations in double, per-population products and
//                relaxation in float on deviations (precision ablation);
//   kDevF32:     float deviations, all arithmetic in float (precision ablation).
constexpr int kF64 = 0, kDevF64 = 1, kDevMixed = 2, kDevF32 = 3;
template <int DT>
using store_t = typename std::conditional<DT == kF64, double, float>::type;

// 1-D weights of c = -1, 0, +1 (Sec. "Basic concepts").
__host__ __device__ constexpr double w1(int k) { return k == 1 ? 2.0 / 3.0 : 1.0 / 6.0; }

// D1Q3, D2Q9 and D3Q27 as tensor products of the 1-D stencil.  Loops over
// (cz, cy, cx) with cy < NY, cz < NZ visit i = cx + 3 cy + 9 cz; the lattice
// velocity along y is cy - 1 when DIM >= 2 (along z likewise when DIM == 3).
template <int DIM>
struct Lattice {
    static constexpr int Q = DIM == 1 ? 3 : (DIM == 2 ? 9 : 27);
    static constexpr int NY = DIM >= 2 ? 3 : 1;  // number of c_y values
    static constexpr int NZ = DIM == 3 ? 3 : 1;  // number of c_z values
    __host__ __device__ static constexpr double weight(int i) {
        return DIM == 1 ? w1(i) : w1(i % 3) * w1((i / 3) % 3) * (DIM == 2 ? 1.0 : w1(i / 9));
    }
};

// Moments of the stored values of one node.  rho_shift = rho0 for deviation
// storage, 0 otherwise.  j is the momentum rho u.
template <int DIM>
__device__ __forceinline__ void node_moments(const double (&f)[Lattice<DIM>::Q], double rho_shift,
                                             double &rho, double (&j)[3]) {
    if constexpr (DIM == 1) {
        rho = rho_shift + ((f[0] + f[1]) + f[2]);
        j[0] = f[2] - f[0];
        j[1] = 0.0;
        j[2] = 0.0;
    } else {
        // Row sums over c_x for every (c_y, c_z), then combine.
        double row[3][3], rowx[3][3];
#pragma unroll
        for (int cz = 0; cz < Lattice<DIM>::NZ; ++cz)
#pragma unroll
            for (int cy = 0; cy < 3; ++cy) {
                const int b = 3 * cy + 9 * cz;
                row[cz][cy] = (f[b + 0] + f[b + 1]) + f[b + 2];
                rowx[cz][cy] = f[b + 2] - f[b + 0];
            }
        double s = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
        for (int cz = 0; cz < Lattice<DIM>::NZ; ++cz) {
            const double plane = (row[cz][0] + row[cz][1]) + row[cz][2];
            s += plane;
            jx += (rowx[cz][0] + rowx[cz][1]) + rowx[cz][2];
            jy += row[cz][2] - row[cz][0];
            if (DIM == 3)
                jz += (cz == 2 ? plane : (cz == 0 ? -plane : 0.0));
        }
        rho = rho_shift + s;
        j[0] = jx;
        j[1] = jy;
        j[2] = jz;
    }
}

// Square root of x on [1, 4), the range of S^2 = 1 + 3 u^2 for |u| < 1.  On the
// device: the hardware estimate of 1/sqrt(x), one coupled Goldschmidt step
// (g -> sqrt(x), h -> 1/(2 sqrt(x))) and two Newton corrections of g with the
// residual x - g^2 taken exactly by a fused multiply-add (P. Markstein,
// "IA-64 and Elementary Functions", 2000, ch. 8; the same scheme as a general
// double square root, without the scaling that inputs near the ends of the
// exponent range need and this range does not).  The result is within one
// unit in the last place.  Outside [1, 4) -- a node that has left the
// equilibrium's domain, flagged anyway -- its value is unspecified.
__host__ __device__ __forceinline__ double sqrt_1to4(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    double d = fma(-g, g, x);
    g = fma(d, h, g);
    d = fma(-g, g, x);
    return fma(d, h, g);
#else
    return sqrt(x);
#endif
}

// 1 / x for the density of a node (x > 0 and of order 1 inside the
// equilibrium's domain): the hardware reciprocal estimate and two
// Newton-Raphson steps r <- r + r (1 - x r), within one unit in the last
// place; for x <= 0 or non-finite (a node outside the domain, flagged) the
// value is unspecified.
__device__ __forceinline__ double recip_density(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// Per-axis equilibrium factors g_{-1}, g_0, g_{+1} and S = sqrt(1 + 3 u^2).
__host__ __device__ __forceinline__ void axis_factors(double u, double (&g)[3], double &S) {
    S = sqrt_1to4(fma(3.0 * u, u, 1.0));
    const double h = fma(2.0, S, -1.0) * (1.0 / 6.0);
    const double half_u = 0.5 * u;
    g[0] = h - half_u;
    g[1] = fma(-2.0, h, 1.0);
    g[2] = h + half_u;
}

// 2 beta with the bulk-viscosity correction at the node's largest |u_a|.
__host__ __device__ __forceinline__ double corrected_omega(double umax, double Smax, double two_tau_m1) {
    const double v2 = 3.0 * umax * umax;
    const double sp1 = Smax + 1.0;
    const double q = 2.0 * (Smax * Smax) * (sp1 * sp1);
    const double p = fma(q, fma(-1.5, v2, 1.0), (v2 * v2) * fma(3.0, sp1 * sp1, 1.0));
    return (2.0 * p) / fma(two_tau_m1, q, p);
}

// Equilibrium kinds (the values of lbm_config.equilibrium).
//   kEqEntropic: eq. (Entropic_isothermal_EDF), the product of the 1-D factors above;
//   kEqPoly2:    eq. (Poly2_isothermal_EDF),
//                w_i rho (1 + c.u / s2 + (c.u)^2 / (2 s2^2) - u^2 / (2 s2)), s2 = 1/3;
//   kEqProduct:  eq. (Product_isothermal_EDF), rho prod_a phi_{c_ia}(u_a) with
//                phi_0 = 1 - s2 - u^2 and phi_{+-1} = (+-u + s2 + u^2) / 2.
constexpr int kEqEntropic = 0, kEqPoly2 = 1, kEqProduct = 2;
// Not an equilibrium: the collision is left out and the populations stream
// unchanged.  Only the measurement of the access pattern's own ceiling uses
// it (lbm_ceiling_stream): the same kernels, loads and stores, no arithmetic.
constexpr int kEqStreamOnly = -1;

// (phi_0 is formed as 1 - (s2 + u^2) so that the factors sum to 1 up to rounding.)
__host__ __device__ __forceinline__ void product_factors(double u, double (&g)[3]) {
    const double base = fma(u, u, 1.0 / 3.0);
    g[0] = (base - u) * 0.5;
    g[1] = 1.0 - base;
    g[2] = (base + u) * 0.5;
}

// 6^D w_i: the lattice weights as integers (1-D: 1, 4, 1).  The second-order
// polynomial equilibrium scales them by rho / 6^D, one correctly rounded
// division per node, so that the weights sum to 1 exactly.
__host__ __device__ constexpr double w1_int(int k) { return k == 1 ? 4.0 : 1.0; }

// 2 beta with the correction for polynomial equilibria, eq. (redefined_relaxation
// rate_poly): A = 1 - (3/2) u^2 / s2 (eq. LBGK_bulk) at the node's largest |u_a|.
// A < 0 beyond |u| = s2^(1/2) (2/3)^(1/2) and beta leaves [0, 1]; nothing is clamped.
__host__ __device__ __forceinline__ double corrected_omega_poly(double umax, double two_tau_m1) {
    const double A = fma(-4.5 * umax, umax, 1.0);
    return (2.0 * A) / (A + two_tau_m1);
}

// Relaxation parameters of a domain.
struct Relax {
    double omega;       // 1 / tau (no correction)
    double two_tau_m1;  // 2 tau - 1 (correction)
    double rho0;        // deviation reference (DEV storage)
};

// One collision of one node: on entry v holds the stored (pre-collision)
// values, on exit the stored post-collision values (rounded to nearest from
// double when the storage is float).  Returns true when the node is outside
// the equilibrium's domain (rho <= 0, |u_a| >= 1 or NaN).  T is the storage
// type; every kernel calls this one function, so a node's result does not
// depend on which kernel or launch shape computed it.
template <int DIM, bool DEV, bool CORR, int EQ = kEqEntropic, typename T>
__device__ __forceinline__ bool collide(T (&v)[Lattice<DIM>::Q], const Relax &r) {
    double f[Lattice<DIM>::Q];
#pragma unroll
    for (int i = 0; i < Lattice<DIM>::Q; ++i)
        f[i] = (double)v[i];
    double rho, j[3];
    node_moments<DIM>(f, DEV ? r.rho0 : 0.0, rho, j);
    const double inv = recip_density(rho);
    double u[3] = {j[0] * inv, j[1] * inv, DIM == 3 ? j[2] * inv : 0.0};
    bool bad = !(rho > 0.0);
#pragma unroll
    for (int a = 0; a < DIM; ++a)
        bad |= !(fabs(u[a]) < 1.0);

    double g[3][3], S[3];
    double usq = 0.0;
    if constexpr (EQ == kEqEntropic) {
#pragma unroll
        for (int a = 0; a < DIM; ++a)
            axis_factors(u[a], g[a], S[a]);
    } else if constexpr (EQ == kEqProduct) {
#pragma unroll
        for (int a = 0; a < DIM; ++a)
            product_factors(u[a], g[a]);
    } else {
#pragma unroll
        for (int a = 0; a < DIM; ++a)
            usq = fma(u[a], u[a], usq);
    }

    double omega = r.omega;
    if (CORR) {
        double umax = fabs(u[0]);
        if constexpr (EQ == kEqEntropic) {
            double Smax = S[0];
#pragma unroll
            for (int a = 1; a < DIM; ++a) {
                umax = fmax(umax, fabs(u[a]));
                Smax = fmax(Smax, S[a]);
            }
            omega = corrected_omega(umax, Smax, r.two_tau_m1);
        } else {
#pragma unroll
            for (int a = 1; a < DIM; ++a)
                umax = fmax(umax, fabs(u[a]));
            omega = corrected_omega_poly(umax, r.two_tau_m1);
        }
    }

    const double base_poly = fma(-1.5, usq, 1.0);
    const double rho_w = EQ == kEqPoly2 ? rho / (DIM == 1 ? 6.0 : (DIM == 2 ? 36.0 : 216.0)) : 0.0;
    const double ux2_45 = (4.5 * u[0]) * u[0];
#pragma unroll
    for (int cz = 0; cz < Lattice<DIM>::NZ; ++cz)
#pragma unroll
        for (int cy = 0; cy < Lattice<DIM>::NY; ++cy) {
            const double t = EQ == kEqPoly2 || DIM == 1
                                 ? rho
                                 : (DIM == 3 ? (rho * g[1][cy]) * g[2][cz] : rho * g[1][cy]);
            // second-order polynomial along the row: with p = c_y u_y + c_z u_z,
            // 1 + 3 c.u + 4.5 (c.u)^2 - 1.5 u^2 = pp + c_x odd + c_x^2 4.5 u_x^2,
            // pp = 1 - 1.5 u^2 + 3 p + 4.5 p^2, odd = 3 u_x (1 + 3 p)
            double pp = 0.0, odd = 0.0, row_w = 0.0;
            if constexpr (EQ == kEqPoly2) {
                const double p = (DIM >= 2 ? (cy - 1) * u[1] : 0.0) + (DIM == 3 ? (cz - 1) * u[2] : 0.0);
                pp = fma(p, fma(4.5, p, 3.0), base_poly);
                odd = (3.0 * u[0]) * fma(3.0, p, 1.0);
                row_w = rho_w * ((DIM >= 2 ? w1_int(cy) : 1.0) * (DIM == 3 ? w1_int(cz) : 1.0));
            }
#pragma unroll
            for (int cx = 0; cx < 3; ++cx) {
                const int i = cx + 3 * cy + 9 * cz;
                double feq;
                if constexpr (EQ == kEqPoly2) {
                    const double P = cx == 1 ? pp : (cx == 2 ? (pp + ux2_45) + odd : (pp + ux2_45) - odd);
                    feq = (w1_int(cx) * row_w) * P;
                } else {
                    feq = t * g[0][cx];
                }
                if (DEV)
                    feq = fma(-Lattice<DIM>::weight(i), r.rho0, feq);
                T vi = v[i];
                if (sizeof(T) == 4)
                    // Widen again rather than keep the first pass's doubles alive:
                    // an empty asm hides vi's origin (no instruction is emitted and
                    // the value is unchanged), halving the registers held here.
                    asm volatile("" : "+v"(vi));
                const double fi = (double)vi;
                v[i] = (T)fma(omega, feq - fi, fi);
            }
        }
    return bad;
}

// Collision on deviation storage with float per-population arithmetic.
// With S = sqrt(1 + 3 u^2) and q = S - 1 = 3 u^2 / (1 + S), each 1-D factor is
// g(c) = w1(c) (1 + d(c)) with d(0) = -q and d(+-1) = 2 q +- 3 u, so
//   f_i^eq - w_i rho0 = w_i [(rho - rho0) + rho P_i],  P_i = prod_a (1 + d_a) - 1,
// and P_i is formed as nested d + e + d e terms: every float operation acts on
// deviation-sized numbers, never on w_i rho0 itself.  F64MOM selects double
// (else float) for the moment sums, the square roots and d.
template <int DIM, bool CORR, bool F64MOM>
__device__ __forceinline__ bool collide_dev_f32(float (&v)[Lattice<DIM>::Q], const Relax &r) {
    using R = typename std::conditional<F64MOM, double, float>::type;
    constexpr int Q = Lattice<DIM>::Q;
    R f[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i)
        f[i] = (R)v[i];
    // moment sums of the deviations (row sums over c_x, then planes)
    R drho = 0, jx = 0, jy = 0, jz = 0;
    if constexpr (DIM == 1) {
        drho = (f[0] + f[1]) + f[2];
        jx = f[2] - f[0];
    } else {
        R row[3][3], rowx[3][3];
#pragma unroll
        for (int cz = 0; cz < Lattice<DIM>::NZ; ++cz)
#pragma unroll
            for (int cy = 0; cy < 3; ++cy) {
                const int b = 3 * cy + 9 * cz;
                row[cz][cy] = (f[b + 0] + f[b + 1]) + f[b + 2];
                rowx[cz][cy] = f[b + 2] - f[b + 0];
            }
#pragma unroll
        for (int cz = 0; cz < Lattice<DIM>::NZ; ++cz) {
            const R plane = (row[cz][0] + row[cz][1]) + row[cz][2];
            drho += plane;
            jx += (rowx[cz][0] + rowx[cz][1]) + rowx[cz][2];
            jy += row[cz][2] - row[cz][0];
            if (DIM == 3)
                jz += (cz == 2 ? plane : (cz == 0 ? -plane : R(0)));
        }
    }
    const R rho = (R)r.rho0 + drho;
    const R inv = R(1) / rho;
    const R u[3] = {jx * inv, DIM >= 2 ? jy * inv : R(0), DIM == 3 ? jz * inv : R(0)};
    bool bad = !(rho > R(0));
#pragma unroll
    for (int a = 0; a < DIM; ++a)
        bad |= !(fabs(u[a]) < R(1));

    float d[3][3];
    R Smax = 0, umax = 0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const R three_u = R(3) * u[a];
        const R S = sqrt(fma(three_u, u[a], R(1)));
        const R q = (three_u * u[a]) / (R(1) + S);
        d[a][0] = (float)fma(R(2), q, -three_u);
        d[a][1] = (float)(-q);
        d[a][2] = (float)fma(R(2), q, three_u);
        Smax = a == 0 ? S : fmax(Smax, S);
        umax = a == 0 ? fabs(u[a]) : fmax(umax, fabs(u[a]));
    }
    float omega = (float)r.omega;
    if (CORR)
        omega = (float)corrected_omega((double)umax, (double)Smax, r.two_tau_m1);

    const float rf = (float)rho, drf = (float)drho;
#pragma unroll
    for (int cz = 0; cz < Lattice<DIM>::NZ; ++cz)
#pragma unroll
        for (int cy = 0; cy < Lattice<DIM>::NY; ++cy) {
            const float e = DIM == 3 ? fmaf(d[1][cy], d[2][cz], d[1][cy] + d[2][cz]) : (DIM == 2 ? d[1][cy] : 0.0f);
#pragma unroll
            for (int cx = 0; cx < 3; ++cx) {
                const int i = cx + 3 * cy + 9 * cz;
                const float P = fmaf(d[0][cx], e, d[0][cx] + e);
                const float feq = (float)Lattice<DIM>::weight(i) * fmaf(rf, P, drf);
                v[i] = fmaf(omega, feq - v[i], v[i]);
            }
        }
    return bad;
}

// Collision of a node for storage/arithmetic code DT.
// (The single-precision ablation modes exist for the entropic equilibrium only.)
template <int DIM, int DT, bool CORR, int EQ = kEqEntropic>
__device__ __forceinline__ bool collide_dt(store_t<DT> (&v)[Lattice<DIM>::Q], const Relax &r) {
    if constexpr (EQ == kEqStreamOnly)
        return false;
    else if constexpr (DT == kDevMixed)
        return collide_dev_f32<DIM, CORR, true>(v, r);
    else if constexpr (DT == kDevF32)
        return collide_dev_f32<DIM, CORR, false>(v, r);
    else
        return collide<DIM, DT != kF64, CORR, EQ>(v, r);
}

// Stored equilibrium of (rho, u) for initialisation; returns the domain flag.
template <int DIM, bool DEV, int EQ = kEqEntropic>
__device__ __forceinline__ bool equilibrium_stored(double rho, const double (&u)[3], double rho0,
                                                   double (&f)[Lattice<DIM>::Q]) {
    bool bad = !(rho > 0.0);
#pragma unroll
    for (int a = 0; a < DIM; ++a)
        bad |= !(fabs(u[a]) < 1.0);
    double g[3][3], S[3];
    double usq = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        if constexpr (EQ == kEqEntropic)
            axis_factors(u[a], g[a], S[a]);
        else if constexpr (EQ == kEqProduct)
            product_factors(u[a], g[a]);
        else
            usq = fma(u[a], u[a], usq);
    }
    const double base_poly = fma(-1.5, usq, 1.0);
    const double rho_w = EQ == kEqPoly2 ? rho / (DIM == 1 ? 6.0 : (DIM == 2 ? 36.0 : 216.0)) : 0.0;
    const double ux2_45 = (4.5 * u[0]) * u[0];
#pragma unroll
    for (int cz = 0; cz < Lattice<DIM>::NZ; ++cz)
#pragma unroll
        for (int cy = 0; cy < Lattice<DIM>::NY; ++cy) {
            const double t = EQ == kEqPoly2 || DIM == 1
                                 ? rho
                                 : (DIM == 3 ? (rho * g[1][cy]) * g[2][cz] : rho * g[1][cy]);
            // second-order polynomial along the row: with p = c_y u_y + c_z u_z,
            // 1 + 3 c.u + 4.5 (c.u)^2 - 1.5 u^2 = pp + c_x odd + c_x^2 4.5 u_x^2,
            // pp = 1 - 1.5 u^2 + 3 p + 4.5 p^2, odd = 3 u_x (1 + 3 p)
            double pp = 0.0, odd = 0.0, row_w = 0.0;
            if constexpr (EQ == kEqPoly2) {
                const double p = (DIM >= 2 ? (cy - 1) * u[1] : 0.0) + (DIM == 3 ? (cz - 1) * u[2] : 0.0);
                pp = fma(p, fma(4.5, p, 3.0), base_poly);
                odd = (3.0 * u[0]) * fma(3.0, p, 1.0);
                row_w = rho_w * ((DIM >= 2 ? w1_int(cy) : 1.0) * (DIM == 3 ? w1_int(cz) : 1.0));
            }
#pragma unroll
            for (int cx = 0; cx < 3; ++cx) {
                const int i = cx + 3 * cy + 9 * cz;
                double feq;
                if constexpr (EQ == kEqPoly2) {
                    const double P = cx == 1 ? pp : (cx == 2 ? (pp + ux2_45) + odd : (pp + ux2_45) - odd);
                    feq = (w1_int(cx) * row_w) * P;
                } else {
                    feq = t * g[0][cx];
                }
                if (DEV)
                    feq = fma(-Lattice<DIM>::weight(i), rho0, feq);
                f[i] = feq;
            }
        }
    return bad;
}

}  // namespace lbm
