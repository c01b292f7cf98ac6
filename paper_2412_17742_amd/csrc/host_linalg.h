// Small dense complex linear algebra for the one-off FP64 state assembly on the
// host (per instance, O(n^3) once; the per-grid-point work runs on the GPU).
#pragma once
#include <cmath>
#include <complex>
#include <vector>

namespace cgd {

using cplx = std::complex<double>;

struct CMat {
    int r = 0, c = 0;
    std::vector<cplx> a;
    CMat() = default;
    CMat(int r_, int c_) : r(r_), c(c_), a((size_t)r_ * c_, cplx(0, 0)) {}
    cplx &operator()(int i, int j) { return a[(size_t)i * c + j]; }
    const cplx &operator()(int i, int j) const { return a[(size_t)i * c + j]; }
    static CMat eye(int n) {
        CMat m(n, n);
        for (int i = 0; i < n; ++i) m(i, i) = 1.0;
        return m;
    }
};

// complex products written out in real arithmetic (std::complex's operator*
// carries a check for inf/nan on every product)
inline CMat matmul(const CMat &A, const CMat &B) {
    CMat C(A.r, B.c);
    for (int i = 0; i < A.r; ++i) {
        double *crow = reinterpret_cast<double *>(&C.a[(size_t)i * C.c]);
        for (int k = 0; k < A.c; ++k) {
            const double ar = A(i, k).real(), ai = A(i, k).imag();
            if (ar == 0.0 && ai == 0.0) continue;
            const double *brow = reinterpret_cast<const double *>(&B.a[(size_t)k * B.c]);
            for (int j = 0; j < B.c; ++j) {
                const double br = brow[2 * j], bi = brow[2 * j + 1];
                crow[2 * j] += ar * br - ai * bi;
                crow[2 * j + 1] += ar * bi + ai * br;
            }
        }
    }
    return C;
}

inline CMat transpose(const CMat &A) {
    CMat T(A.c, A.r);
    for (int i = 0; i < A.r; ++i)
        for (int j = 0; j < A.c; ++j) T(j, i) = A(i, j);
    return T;
}

inline CMat conj(const CMat &A) {
    CMat T(A.r, A.c);
    for (size_t i = 0; i < A.a.size(); ++i) T.a[i] = std::conj(A.a[i]);
    return T;
}

inline CMat adjoint(const CMat &A) { return conj(transpose(A)); }

// LU with partial pivoting in place; returns false if singular.  perm[i] is
// the original row now at position i; sign is the permutation parity.
inline bool lu_pivoted(CMat &A, std::vector<int> &perm, int &sign) {
    const int n = A.r;
    perm.resize(n);
    for (int i = 0; i < n; ++i) perm[i] = i;
    sign = 1;
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = std::abs(A(k, k));
        for (int i = k + 1; i < n; ++i)
            if (std::abs(A(i, k)) > best) { best = std::abs(A(i, k)); p = i; }
        if (best == 0.0) return false;
        if (p != k) {
            for (int j = 0; j < n; ++j) std::swap(A(k, j), A(p, j));
            std::swap(perm[k], perm[p]);
            sign = -sign;
        }
        const cplx inv = 1.0 / A(k, k);
        for (int i = k + 1; i < n; ++i) {
            const cplx l = A(i, k) * inv;
            A(i, k) = l;
            if (l == cplx(0, 0)) continue;
            for (int j = k + 1; j < n; ++j) A(i, j) -= l * A(k, j);
        }
    }
    return true;
}

// Solve A X = B (A square) by pivoted LU; returns false if singular.
inline bool solve(const CMat &A, const CMat &B, CMat &X) {
    CMat LU = A;
    std::vector<int> perm;
    int sign;
    if (!lu_pivoted(LU, perm, sign)) return false;
    const int n = A.r, m = B.c;
    X = CMat(n, m);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < m; ++j) X(i, j) = B(perm[i], j);
    for (int k = 0; k < n; ++k)
        for (int i = k + 1; i < n; ++i) {
            const cplx l = LU(i, k);
            if (l == cplx(0, 0)) continue;
            for (int j = 0; j < m; ++j) X(i, j) -= l * X(k, j);
        }
    for (int k = n - 1; k >= 0; --k) {
        const cplx inv = 1.0 / LU(k, k);
        for (int j = 0; j < m; ++j) X(k, j) *= inv;
        for (int i = 0; i < k; ++i) {
            const cplx u = LU(i, k);
            if (u == cplx(0, 0)) continue;
            for (int j = 0; j < m; ++j) X(i, j) -= u * X(k, j);
        }
    }
    return true;
}

inline bool inverse(const CMat &A, CMat &Ainv) { return solve(A, CMat::eye(A.r), Ainv); }

// Cholesky test of a Hermitian matrix: true iff numerically positive definite.
inline bool hermitian_positive_definite(const CMat &A) {
    const int n = A.r;
    CMat L(n, n);
    for (int j = 0; j < n; ++j) {
        double d = A(j, j).real();
        for (int k = 0; k < j; ++k) d -= std::norm(L(j, k));
        if (!(d > 0.0)) return false;
        const double ljj = std::sqrt(d);
        L(j, j) = ljj;
        for (int i = j + 1; i < n; ++i) {
            cplx s = A(i, j);
            for (int k = 0; k < j; ++k) s -= L(i, k) * std::conj(L(j, k));
            L(i, j) = s / ljj;
        }
    }
    return true;
}

// log det of a Hermitian positive definite matrix (via Cholesky); NaN if not PD.
inline double logdet_hpd(const CMat &A) {
    const int n = A.r;
    CMat L(n, n);
    double acc = 0.0;
    for (int j = 0; j < n; ++j) {
        double d = A(j, j).real();
        for (int k = 0; k < j; ++k) d -= std::norm(L(j, k));
        if (!(d > 0.0)) return NAN;
        const double ljj = std::sqrt(d);
        acc += 2.0 * std::log(ljj);
        L(j, j) = ljj;
        for (int i = j + 1; i < n; ++i) {
            cplx s = A(i, j);
            for (int k = 0; k < j; ++k) s -= L(i, k) * std::conj(L(j, k));
            L(i, j) = s / ljj;
        }
    }
    return acc;
}

// Eigen-decomposition of a Hermitian matrix by cyclic complex Jacobi
// rotations: A = V diag(lam) V^H, V unitary.  Returns false if it did not
// converge.
inline bool hermitian_eig(const CMat &Ain, std::vector<double> &lam, CMat &V) {
    const int n = Ain.r;
    CMat A = Ain;
    V = CMat::eye(n);
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                tot += std::norm(A(i, j));
                if (i != j) off += std::norm(A(i, j));
            }
        if (off <= 1e-30 * (tot + 1e-300)) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const cplx apq = A(p, q);
                const double g = std::abs(apq);
                if (g < 1e-300) continue;
                const double app = A(p, p).real(), aqq = A(q, q).real();
                // rotate in the (p,q) plane: with apq = g e^{i phi}, the real
                // symmetric 2x2 [[app, g],[g, aqq]] is diagonalised by angle t
                const cplx e = apq / g;  // e^{i phi}
                const double theta = 0.5 * std::atan2(2.0 * g, aqq - app);
                const double c = std::cos(theta), s = std::sin(theta);
                // columns p, q of the rotation R: R(p,p)=c, R(q,p)=-s e^{-i phi},
                // R(p,q)= s e^{i phi}, R(q,q)=c   (A <- R^H A R)
                const cplx rpq = s * e, rqp = -s * std::conj(e);
                for (int k = 0; k < n; ++k) {  // A <- A R (columns)
                    const cplx akp = A(k, p), akq = A(k, q);
                    A(k, p) = akp * c + akq * rqp;
                    A(k, q) = akp * rpq + akq * c;
                }
                for (int k = 0; k < n; ++k) {  // A <- R^H A (rows)
                    const cplx apk = A(p, k), aqk = A(q, k);
                    A(p, k) = c * apk + std::conj(rqp) * aqk;
                    A(q, k) = std::conj(rpq) * apk + c * aqk;
                }
                A(p, q) = 0.0;
                A(q, p) = 0.0;
                A(p, p) = A(p, p).real();
                A(q, q) = A(q, q).real();
                for (int k = 0; k < n; ++k) {  // V <- V R
                    const cplx vkp = V(k, p), vkq = V(k, q);
                    V(k, p) = vkp * c + vkq * rqp;
                    V(k, q) = vkp * rpq + vkq * c;
                }
            }
        if (sweep == 99) return false;
    }
    lam.resize(n);
    for (int i = 0; i < n; ++i) lam[i] = A(i, i).real();
    return true;
}

}  // namespace cgd
