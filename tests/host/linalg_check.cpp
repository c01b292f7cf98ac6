// Test driver for the host linear algebra of the library (host_linalg.h):
// reads a Hermitian matrix (n, then n*n complex entries as re im pairs,
// row-major, binary doubles) from argv[1], writes to argv[2] the eigenvalues
// and eigenvectors of hermitian_eig_ql, the eigenvalues of hermitian_eigvals,
// and the tridiagonal form (d, e) of hermitian_tridiag.
#include <cstdio>
#include <vector>

#include "../../paper_2412_17742_amd/csrc/host_linalg.h"

using namespace cgd;

int main(int argc, char **argv) {
    if (argc != 3) return 2;
    FILE *f = std::fopen(argv[1], "rb");
    if (!f) return 3;
    double nd = 0;
    if (std::fread(&nd, sizeof(double), 1, f) != 1) return 4;
    const int n = (int)nd;
    CMat A(n, n);
    if (std::fread(A.a.data(), sizeof(cplx), (size_t)n * n, f) != (size_t)n * n) return 5;
    std::fclose(f);
    std::vector<double> lam, lam2, d, e;
    CMat V;
    const bool ok1 = hermitian_eig_ql(A, lam, V);
    const bool ok2 = hermitian_eigvals(A, lam2);
    hermitian_tridiag(A, d, e, nullptr);
    // a solver that gave up leaves its outputs empty: write zeros after the flags
    lam.resize(n, 0.0);
    lam2.resize(n, 0.0);
    if (V.r != n) V = CMat(n, n);
    FILE *o = std::fopen(argv[2], "wb");
    if (!o) return 6;
    const double flags[2] = {(double)ok1, (double)ok2};
    std::fwrite(flags, sizeof(double), 2, o);
    std::fwrite(lam.data(), sizeof(double), n, o);
    std::fwrite(V.a.data(), sizeof(cplx), (size_t)n * n, o);
    std::fwrite(lam2.data(), sizeof(double), n, o);
    std::fwrite(d.data(), sizeof(double), n, o);
    std::fwrite(e.data(), sizeof(double), n, o);
    std::fclose(o);
    return 0;
}
