// Host run of the GPU eigensolver header (csrc/vn.hpp): builds the
// amplification matrix of each case, reduces it to Hessenberg form and
// iterates QR steps one matrix at a time (the group of lockstep threads is the
// thread itself, and the reciprocal square root estimate is the host stand-in).
// Usage: vn_host <dim 1|2> <equilibrium 0|1|2> <correction 0|1> <in> <out>
// in: int64 count, then count x 5 doubles (tau, u_x, u_y, k_x, k_y);
// out: count x N complex eigenvalues (re, im doubles), then count int32 QR step counts.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "vn.hpp"

using namespace lbm;

template <int DIM, int EQ, bool CORR>
static void run(const std::vector<double> &c, std::vector<double> &eig, std::vector<int> &steps) {
    constexpr int N = DIM == 1 ? 3 : 9;
    const size_t n = c.size() / 5;
    for (size_t t = 0; t < n; ++t) {
        const double *p = &c[5 * t];
        const double u[2] = {p[1], DIM == 2 ? p[2] : 0.0}, k[2] = {p[3], DIM == 2 ? p[4] : 0.0};
        cplx H[N][N];
        vn_matrix<DIM, EQ, CORR>(p[0], u, k, H);
        hessenberg<N>(H);
        steps[t] = hessenberg_eigenvalues<N>(H, [](int v) { return v; });
        for (int i = 0; i < N; ++i) {
            eig[(t * N + i) * 2] = H[i][i].re;
            eig[(t * N + i) * 2 + 1] = H[i][i].im;
        }
    }
}

template <int DIM, int EQ>
static void run_c(bool corr, const std::vector<double> &c, std::vector<double> &eig, std::vector<int> &steps) {
    if (corr)
        run<DIM, EQ, true>(c, eig, steps);
    else
        run<DIM, EQ, false>(c, eig, steps);
}

template <int DIM>
static void run_eq(int eq, bool corr, const std::vector<double> &c, std::vector<double> &eig,
                   std::vector<int> &steps) {
    if (eq == kEqPoly2)
        run_c<DIM, kEqPoly2>(corr, c, eig, steps);
    else if (eq == kEqProduct)
        run_c<DIM, kEqProduct>(corr, c, eig, steps);
    else
        run_c<DIM, kEqEntropic>(corr, c, eig, steps);
}

int main(int argc, char **argv) {
    if (argc != 6)
        return 2;
    const int dim = atoi(argv[1]), eq = atoi(argv[2]), corr = atoi(argv[3]);
    FILE *f = fopen(argv[4], "rb");
    long long n = 0;
    if (!f || fread(&n, 8, 1, f) != 1 || n < 0)
        return 3;
    std::vector<double> c(5 * n);
    if (fread(c.data(), 8, c.size(), f) != c.size())
        return 3;
    fclose(f);
    const int N = dim == 1 ? 3 : 9;
    std::vector<double> eig(2 * N * n);
    std::vector<int> steps(n);
    if (dim == 1)
        run_eq<1>(eq, corr != 0, c, eig, steps);
    else
        run_eq<2>(eq, corr != 0, c, eig, steps);
    FILE *g = fopen(argv[5], "wb");
    if (!g || fwrite(eig.data(), 8, eig.size(), g) != eig.size() ||
        fwrite(steps.data(), 4, steps.size(), g) != steps.size())
        return 4;
    fclose(g);
    return 0;
}
