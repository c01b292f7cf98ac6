// Small dense complex linear algebra for the one-off FP64 state assembly on the
// host (per instance, O(n^3) once; the per-grid-point work runs on the GPU).
#pragma once
#include <algorithm>
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

// Householder reduction of a Hermitian matrix to real symmetric tridiagonal
// form: A = Q D T D^H Q^H with Q a product of Householder reflectors, D a
// diagonal of unit phases and T real (diagonal d, subdiagonal e >= 0, e[n-1]
// unused).  With Q (and D folded into it) kept when want_q: Qd = Q D.
inline void hermitian_tridiag(const CMat &Ain, std::vector<double> &d, std::vector<double> &e, CMat *Qd) {
    const int n = Ain.r;
    CMat A = Ain;
    d.assign(n, 0.0);
    e.assign(n, 0.0);
    std::vector<cplx> v(n), p(n), beta(n, cplx(0, 0));
    if (Qd) *Qd = CMat::eye(n);
    for (int k = 0; k + 2 < n; ++k) {
        // reflector H = I - tau v v^H zeroing A[k+2.., k]
        double xn2 = 0;
        for (int i = k + 1; i < n; ++i) xn2 += std::norm(A(i, k));
        const double xn = std::sqrt(xn2);
        const cplx x0 = A(k + 1, k);
        const double ax0 = std::abs(x0);
        if (xn == 0.0 || xn2 - ax0 * ax0 <= 1e-300 * (xn2 + 1e-300)) {
            beta[k] = x0;  // already zero below the subdiagonal
            continue;
        }
        const cplx ph = ax0 > 0 ? x0 / ax0 : cplx(1, 0);
        const cplx alpha = -ph * xn;  // H x = alpha e_1
        for (int i = 0; i < n; ++i) v[i] = 0.0;
        v[k + 1] = x0 - alpha;
        for (int i = k + 2; i < n; ++i) v[i] = A(i, k);
        double vn2 = 0;
        for (int i = k + 1; i < n; ++i) vn2 += std::norm(v[i]);
        const double tau = 2.0 / vn2;
        // p = tau A v over the trailing block, K = tau/2 v^H p, q = p - K v
        const double *vr = reinterpret_cast<const double *>(v.data());
        for (int i = k + 1; i < n; ++i) {
            const double *ar = reinterpret_cast<const double *>(&A.a[(size_t)i * n]);
            double sr = 0, si = 0;
            for (int j = k + 1; j < n; ++j) {
                sr += ar[2 * j] * vr[2 * j] - ar[2 * j + 1] * vr[2 * j + 1];
                si += ar[2 * j] * vr[2 * j + 1] + ar[2 * j + 1] * vr[2 * j];
            }
            p[i] = cplx(tau * sr, tau * si);
        }
        cplx vp(0, 0);
        for (int i = k + 1; i < n; ++i) vp += std::conj(v[i]) * p[i];
        const double K = 0.5 * tau * vp.real();
        for (int i = k + 1; i < n; ++i) p[i] -= K * v[i];
        // A <- A - v q^H - q v^H on the trailing block; column k becomes alpha e_1
        const double *pr = reinterpret_cast<const double *>(p.data());
        for (int i = k + 1; i < n; ++i) {
            double *ar = reinterpret_cast<double *>(&A.a[(size_t)i * n]);
            const double vi_r = vr[2 * i], vi_i = vr[2 * i + 1], pi_r = pr[2 * i], pi_i = pr[2 * i + 1];
            for (int j = k + 1; j < n; ++j) {
                // v_i conj(p_j) + p_i conj(v_j)
                const double pj_r = pr[2 * j], pj_i = pr[2 * j + 1], vj_r = vr[2 * j], vj_i = vr[2 * j + 1];
                ar[2 * j] -= vi_r * pj_r + vi_i * pj_i + pi_r * vj_r + pi_i * vj_i;
                ar[2 * j + 1] -= vi_i * pj_r - vi_r * pj_i + pi_i * vj_r - pi_r * vj_i;
            }
        }
        beta[k] = alpha;
        for (int i = k + 2; i < n; ++i) A(i, k) = A(k, i) = 0.0;
        A(k + 1, k) = alpha;
        A(k, k + 1) = std::conj(alpha);
        if (Qd) {  // Q <- Q H
            CMat &Q = *Qd;
            for (int r = 0; r < n; ++r) {
                double *qr = reinterpret_cast<double *>(&Q.a[(size_t)r * n]);
                double sr = 0, si = 0;
                for (int j = k + 1; j < n; ++j) {
                    sr += qr[2 * j] * vr[2 * j] - qr[2 * j + 1] * vr[2 * j + 1];
                    si += qr[2 * j] * vr[2 * j + 1] + qr[2 * j + 1] * vr[2 * j];
                }
                sr *= tau;
                si *= tau;
                for (int j = k + 1; j < n; ++j) {  // Q_rj -= s conj(v_j)
                    qr[2 * j] -= sr * vr[2 * j] + si * vr[2 * j + 1];
                    qr[2 * j + 1] -= si * vr[2 * j] - sr * vr[2 * j + 1];
                }
            }
        }
    }
    if (n >= 2) beta[n - 2] = A(n - 1, n - 2);
    for (int i = 0; i < n; ++i) d[i] = A(i, i).real();
    // unit phases ph_0 = 1, ph_{i+1} = ph_i beta_i / |beta_i| make the subdiagonal real
    std::vector<cplx> ph(n, cplx(1, 0));
    for (int i = 0; i + 1 < n; ++i) {
        const double b = std::abs(beta[i]);
        e[i] = b;
        ph[i + 1] = b > 0 ? ph[i] * beta[i] / b : ph[i];
    }
    if (Qd)
        for (int r = 0; r < n; ++r)
            for (int j = 0; j < n; ++j) (*Qd)(r, j) *= ph[j];
}

// Eigenvalues (and, with Z, eigenvectors) of a real symmetric tridiagonal
// matrix (diagonal d, subdiagonal e) by the implicit QL method with Wilkinson
// shifts; Z (n x n, row-major, initialised by the caller) accumulates the
// rotations.  Returns false if an eigenvalue takes more than 60 iterations.
inline bool tridiag_ql(std::vector<double> &d, std::vector<double> e, std::vector<double> *Z) {
    const int n = (int)d.size();
    // a subdiagonal entry is negligible next to its two diagonal neighbours, or
    // at rounding level of the matrix norm (half an ulp, as in EISPACK's tql2):
    // rotations through the large eigenvalues keep about that much noise in the
    // entries of a cluster of eigenvalues near zero (a matrix of low rank), which
    // the relative test alone never accepts
    double anorm = 0.0;
    for (int i = 0; i < n; ++i) anorm = std::max(anorm, std::fabs(d[i]) + (i + 1 < n ? std::fabs(e[i]) : 0.0));
    const double floor_e = 1.1102230246251565e-16 * anorm;
    for (int l = 0; l < n; ++l) {
        int iter = 0;
        for (;;) {
            int m = l;
            for (; m + 1 < n; ++m) {
                const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) <= 1e-16 * dd || std::fabs(e[m]) <= floor_e) break;
            }
            if (m == l) break;
            if (++iter > 60) return false;
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = std::hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
            double s = 1.0, c = 1.0, p = 0.0;
            int i = m - 1;
            for (; i >= l; --i) {
                double f = s * e[i], b = c * e[i];
                r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {
                    d[i + 1] -= p;
                    e[m] = 0.0;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0 * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
                if (Z)
                    for (int k = 0; k < n; ++k) {
                        double &zk1 = (*Z)[(size_t)k * n + i + 1], &zk = (*Z)[(size_t)k * n + i];
                        f = zk1;
                        zk1 = s * zk + c * f;
                        zk = c * zk - s * f;
                    }
            }
            if (r == 0.0 && i >= l) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    return true;
}

// Eigen-decomposition of a Hermitian matrix, A = V diag(lam) V^H: Householder
// tridiagonalisation, then implicit QL on the real tridiagonal form, the
// eigenvectors carried back through the reflectors.  Returns false if QL did
// not converge.
inline bool hermitian_eig_ql(const CMat &A, std::vector<double> &lam, CMat &V) {
    const int n = A.r;
    std::vector<double> d, e;
    CMat Qd;
    hermitian_tridiag(A, d, e, &Qd);
    std::vector<double> Z((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Z[(size_t)i * n + i] = 1.0;
    if (!tridiag_ql(d, e, &Z)) return false;
    lam = d;
    V = CMat(n, n);
    for (int r = 0; r < n; ++r) {
        double *vrow = reinterpret_cast<double *>(&V.a[(size_t)r * n]);
        for (int k = 0; k < n; ++k) {
            const double qr = Qd(r, k).real(), qi = Qd(r, k).imag();
            if (qr == 0.0 && qi == 0.0) continue;
            const double *zr = &Z[(size_t)k * n];
            for (int j = 0; j < n; ++j) {
                vrow[2 * j] += qr * zr[j];
                vrow[2 * j + 1] += qi * zr[j];
            }
        }
    }
    return true;
}

// Eigenvalues only (tridiagonal form and QL, no vectors).
inline bool hermitian_eigvals(const CMat &A, std::vector<double> &lam) {
    std::vector<double> e;
    hermitian_tridiag(A, lam, e, nullptr);
    return tridiag_ql(lam, e, nullptr);
}

}  // namespace cgd
