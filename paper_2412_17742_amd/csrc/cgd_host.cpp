// Host side of the C ABI: validation, FP64 state assembly (once per
// instance), device layout of the per-point factorisation jobs, and the launch
// sequence of an evaluation.  All per-grid-point work runs in the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <thread>
#include <vector>

#include "../../include/cgd.h"
#include "cgd_internal.h"
#include "host_linalg.h"

using namespace cgd;

namespace {

// Mixed path: model of the relative error of an FP32 value of G, per internal
// block of order n: tau = kTauScale (n + 1) 2^-24 (the first-order change of
// log det under the backward error of an n-step unpivoted elimination of an
// accretive matrix stored in FP32, log accumulated in FP64).  Measured on every
// grid point of five workloads, the largest relative error was 0.56 tau; the
// mixed-path tests check the model on workloads with other seeds and shapes.
// The autotuner checks it again on its sample of each context's FP32 items and
// scales tau up wherever the sample's largest error exceeds kTauMargin tau.
constexpr double kTauScale = 2.0;
constexpr double kTauMargin = 0.5;

// moments mode: default number of points per axis on the circle in t
constexpr int kMomentPoints = 24;

thread_local std::string g_err;

cgd_status fail(cgd_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

#define HIP_OK(expr)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(CGD_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Per-block product of the host assembly.
struct HostBlock {
    int inst = 0, blk = 0;
    int nb = 0;                 // order of the matrix factorised per point
    int bordered = 0;
    int nkeep = 0;              // density mode: kept-mode border rows (before the gamma border)
    std::vector<int32_t> kv;    // their generating-function variable positions
    std::vector<int32_t> rowbin;
    CMat H;                     // nb x nb: the matrix itself, or H_BB under elimination
    int schur_axis = -1;        // eliminated bin
    std::vector<double> eig;    // its eigenvalues
    CMat P, Q;                  // H_BA V and V^H H_AB
    int lowrank = 0;            // > 0: rank of H (low-rank route, no factorisation per point)
    std::vector<cplx> lr;       // then G_g = diag(lambda) V^H E_g V, g = traced rows, bins 0..L-1
};

// Gradient data of one internal block: the full (bordered) matrix before any
// reduction, and what the chain rule needs.
struct GradHost {
    int inst = 0, k = 0;
    int n2 = 0, bordered = 0;
    CMat Sinv;                  // Sigma^-1 (2M x 2M)
    std::vector<cplx> v;        // Sigma^-1 zbar
    CMat Hf;                    // bordered H (order n2 + bordered)
    std::vector<int32_t> rb;    // row bins of Hf
};

// Copy of one instance's inputs (the chain rule needs them after create).
struct HostInstCopy {
    int M = 0, K = 1;
    std::vector<cplx> T, alpha_v;
    const cplx *alpha = nullptr;
    std::vector<double> r, schmidt;
    std::vector<std::vector<double>> rk;
};

// Marginal moment generating function of one bin's count within one
// internal block (Sec. VI C, Eq. M, with the other bins' variables at t = 0):
// with R the bin's rows and columns of Sigma - I (the s = 1 ordered covariance)
// and zbar its means, E[s^b] = exp(1/2 u zbar^H (I - u R)^-1 zbar) /
// sqrt(det(I - u R)), u = s - 1.  R is kept as a real tridiagonal T (d, e)
// unitarily similar to it, zbar as z = Q^H zbar in the same basis.
struct BinMarginal {
    std::vector<double> d, e;
    std::vector<cplx> z;  // empty when undisplaced
};

struct HostInst {
    int L = 1;
    int G[kMaxBins] = {0}, N[kMaxBins] = {0};
    bool auto_grid[kMaxBins] = {};
    double logpr0 = 0.0;
    int nblocks = 0;
    std::vector<BinMarginal> marg[kMaxBins];  // per bin, one entry per internal block
    double wrap_bound = 0.0;                   // sum_l bound on Pr(b_l >= G_l)
    double hnorm = 0.0;                        // moments mode: max over blocks of ||I - Sigma^-1||_2
    double rho = 0.0;                          // moments mode: radius of the circle in t
    int nvar = 0, fock_n = 0;                  // density mode: 2 g variables, Fock cutoff
};

// log E[s^b] of a bin, u = s - 1 >= 0, summed over its blocks; +inf outside
// the domain of convergence (I - u T not positive definite).
double bin_log_mgf(const std::vector<BinMarginal> &mb, double u) {
    double acc = 0.0;
    std::vector<double> piv, yr, yi;
    for (const BinMarginal &m : mb) {
        const int n = (int)m.d.size();
        piv.resize(n);
        // LDL^T of the tridiagonal I - u T: pivots must stay positive
        for (int i = 0; i < n; ++i) {
            double p = 1.0 - u * m.d[i];
            if (i > 0) {
                const double o = u * m.e[i - 1];
                p -= o * o / piv[i - 1];
            }
            if (!(p > 0.0)) return INFINITY;
            piv[i] = p;
            acc -= 0.5 * std::log(p);
        }
        if (!m.z.empty()) {
            // y = (I - u T)^-1 z by the same factors (T real: real and imaginary parts apart)
            yr.resize(n);
            yi.resize(n);
            for (int i = 0; i < n; ++i) {
                yr[i] = m.z[i].real();
                yi[i] = m.z[i].imag();
                if (i > 0) {
                    const double l = -u * m.e[i - 1] / piv[i - 1];
                    yr[i] -= l * yr[i - 1];
                    yi[i] -= l * yi[i - 1];
                }
            }
            for (int i = n - 1; i >= 0; --i) {
                yr[i] /= piv[i];
                yi[i] /= piv[i];
                if (i + 1 < n) {
                    const double l = -u * m.e[i] / piv[i];
                    yr[i] -= l * yr[i + 1];
                    yi[i] -= l * yi[i + 1];
                }
            }
            double q = 0.0;
            for (int i = 0; i < n; ++i) q += m.z[i].real() * yr[i] + m.z[i].imag() * yi[i];
            acc += 0.5 * u * q;
        }
    }
    return acc;
}

// log of the Chernoff bound Pr(b >= G) <= min over s > 1 of E[s^b] / s^G: the
// exponent log E[s^b] - G log s is convex in t = log s, minimised by golden
// section over (0, t_max), t_max the edge of convergence (found by doubling
// and bisection) or, when E[s^b] is finite up to s = 1 + 2^60 (a bin without
// squeezed or thermal light: coherent light only, or no light), log(1 + 2^60).
// 0 means no bound below 1.
double bin_log_tail(const std::vector<BinMarginal> &mb, int G) {
    double hi = 1.0, lo = 0.0;
    int it = 0;
    while (it < 60 && std::isfinite(bin_log_mgf(mb, hi))) {
        lo = hi;
        hi *= 2.0;
        ++it;
    }
    if (std::isfinite(bin_log_mgf(mb, hi))) {
        lo = hi;
    } else {
        for (int k = 0; k < 100; ++k) {
            const double mid = 0.5 * (lo + hi);
            (std::isfinite(bin_log_mgf(mb, mid)) ? lo : hi) = mid;
        }
    }
    const double tmax = std::log1p(lo);
    auto f = [&](double t) { return bin_log_mgf(mb, std::expm1(t)) - G * t; };
    const double gr = 0.5 * (std::sqrt(5.0) - 1.0);
    double a = 0.0, b = tmax;
    double x1 = b - gr * (b - a), x2 = a + gr * (b - a), f1 = f(x1), f2 = f(x2);
    for (int k = 0; k < 200 && b - a > 1e-12 * (1.0 + b); ++k) {
        if (f1 <= f2) {
            b = x2;
            x2 = x1;
            f2 = f1;
            x1 = b - gr * (b - a);
            f1 = f(x1);
        } else {
            a = x1;
            x1 = x2;
            f1 = f2;
            x2 = a + gr * (b - a);
            f2 = f(x2);
        }
    }
    return std::min(0.0, std::min(f1, f2));
}

cplx cx(const double *p, size_t i) { return cplx(p[2 * i], p[2 * i + 1]); }

// Largest eigenvalue of T^H T (||T||_2^2).
bool spectral_norm_sq(const double *T, int M, double &out) {
    CMat A(M, M);
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < M; ++j) A(i, j) = cx(T, (size_t)i * M + j);
    CMat G = matmul(adjoint(A), A);
    std::vector<double> lam;
    if (!hermitian_eigvals(G, lam)) return false;
    out = *std::max_element(lam.begin(), lam.end());
    return true;
}

// Rows [0, 2m) of a block: mode index within the block -> bin.
int bin_of_row(const cgd_instance &in, int row, int m, const std::vector<int> &kset, bool dense) {
    const int mode = row % m;
    int i, k;
    if (dense) { i = mode / in.K; k = mode % in.K; }
    else { i = mode; k = kset[0]; }
    return in.resolve_internal ? in.bin_of[i * in.K + k] : in.bin_of[i];
}

// Fine indices i*K + k of the kept modes, ascending (the order of the density
// matrix's multi-indices).
std::vector<int> kept_fine_modes(const cgd_instance &in) {
    std::vector<int> out;
    for (int i = 0; i < in.M; ++i)
        for (int k = 0; k < in.K; ++k) {
            const int b = in.resolve_internal ? in.bin_of[i * in.K + k] : in.bin_of[i];
            if (b == CGD_KEEP) out.push_back(i * in.K + k);
        }
    return out;
}

cgd_status validate(const cgd_instance &in, int idx) {
    const std::string at = "instance " + std::to_string(idx) + ": ";
    if (in.M < 1 || in.K < 1 || in.L < 1 || in.L > kMaxBins) return fail(CGD_ERR_ARG, at + "need M >= 1, K >= 1, 1 <= L <= 8");
    // M internal blocks of order 2M when the inputs are distinguishable, else K of order 2M (or one of 2MK)
    if (in.distinguishable ? in.M > 512 : (int64_t)in.M * in.K > 4096)
        return fail(CGD_ERR_ARG, at + (in.distinguishable ? "M > 512 with distinguishable inputs" : "M*K too large"));
    if (!in.T || !in.r || !in.bin_of || !in.cutoff) return fail(CGD_ERR_ARG, at + "T, r, bin_of and cutoff are required");
    if (in.distinguishable) {
        if (in.K != in.M || in.schmidt || in.alpha)
            return fail(CGD_ERR_ARG, at + "distinguishable inputs need K == M and no schmidt or alpha");
    } else if (in.K > 1 && !in.schmidt) {
        return fail(CGD_ERR_ARG, at + "schmidt weights required when K > 1");
    }
    for (int i = 0; i < in.M * in.M * 2; ++i)
        if (!std::isfinite(in.T[i])) return fail(CGD_ERR_ARG, at + "T not finite");
    for (int i = 0; i < in.M; ++i) {
        if (!std::isfinite(in.r[i]) || in.r[i] < 0) return fail(CGD_ERR_NONPHYSICAL, at + "squeezing must be finite and >= 0");
        if (in.r[i] > 12.0) return fail(CGD_ERR_ARG, at + "squeezing above 12 is not supported");
    }
    if (in.alpha)
        for (int i = 0; i < 2 * in.M; ++i)
            if (!std::isfinite(in.alpha[i])) return fail(CGD_ERR_ARG, at + "alpha not finite");
    if (in.schmidt) {
        double s = 0;
        for (int k = 0; k < in.K; ++k) {
            if (!(in.schmidt[k] > 0) || !std::isfinite(in.schmidt[k])) return fail(CGD_ERR_NONPHYSICAL, at + "schmidt weights must be > 0");
            if (in.schmidt[k] > in.schmidt[0] * (1 + 1e-12)) return fail(CGD_ERR_NONPHYSICAL, at + "schmidt weight above lambda_0");
            s += in.schmidt[k];
        }
        if (std::fabs(s - 1.0) > 1e-9) return fail(CGD_ERR_NONPHYSICAL, at + "schmidt weights must sum to 1");
    }
    const int nbin = in.resolve_internal ? in.M * in.K : in.M;
    for (int i = 0; i < nbin; ++i)
        if (in.bin_of[i] < CGD_KEEP || in.bin_of[i] >= in.L) return fail(CGD_ERR_ARG, at + "bin index out of range");
    const int g = (int)kept_fine_modes(in).size();
    if (g > 0) {
        if (2 * g > kMaxKeepVars) return fail(CGD_ERR_ARG, at + "at most 8 kept modes");
        if (in.fock_cutoff < 0) return fail(CGD_ERR_ARG, at + "fock_cutoff must be >= 0");
        double e = 1.0;
        for (int k = 0; k < 2 * g; ++k) e *= (double)in.fock_cutoff + 1.0;
        if (e > (double)(1 << 22)) return fail(CGD_ERR_ARG, at + "(fock_cutoff + 1)^(2 g) exceeds 2^22");
    }
    int64_t npts = 1;
    for (int l = 0; l < in.L; ++l) {
        if (in.cutoff[l] < 0 || in.cutoff[l] > 4095) return fail(CGD_ERR_ARG, at + "cutoff out of range");
        const int g = in.grid ? in.grid[l] : in.cutoff[l] + 1;
        if (g == 0 && in.grid) continue;  // automatic: chosen from the tail bound
        if (g < in.cutoff[l] + 1 || g > 4096)
            return fail(CGD_ERR_ARG, at + "grid must satisfy cutoff+1 <= G <= 4096 (or 0: automatic)");
        npts *= g;
        if (npts > (int64_t)1 << 31) return fail(CGD_ERR_ARG, at + "grid too large");
    }
    double nrm2;
    if (!spectral_norm_sq(in.T, in.M, nrm2)) return fail(CGD_ERR_NUMERIC, at + "norm of T did not converge");
    if (nrm2 > 1.0 + 1e-10) return fail(CGD_ERR_NONPHYSICAL, at + "||T||_2 > 1");
    return CGD_OK;
}

// Low-rank blocks.  With q squeezed inputs in internal mode k and no
// displacement, Sigma - I = Y C Y^H (Sec. II moments): Y has the columns
// a_j = (t_j, 0) and b_j = (0, conj t_j) for every squeezed input j (t_j:
// column j of T) and C is block diagonal with [[sinh^2, sinh cosh], [sinh cosh,
// sinh^2]] of r_jk per input.  H = I - Sigma^-1 then has rank r = 2q, and
// with |Y| = (Y^H Y)^1/2 and Z = |Y| C |Y| = W diag(z) W^H (order r):
//   H = V diag(z / (1 + z)) V^H,  V = Y |Y|^-1 W (orthonormal columns),
//   log det Sigma = sum log(1 + z),  Sigma > I/2  <=>  z > -1/2,
// and a bin's marginal Y_b C Y_b^H has the nonzero spectrum of |Y_b| C |Y_b|.
// det(I - D H) = det(I_r - diag(lambda) V^H D V) (Sylvester), D constant over
// the rows of a bin (1 on the traced rows), so per point the block's factor is
// the r x r determinant of I - (G_t + sum_l w_l G_l), G_g = diag(lambda) V^H
// E_g V (E_g: the rows of bin g, or the traced rows).  Everything here costs
// O(M r^2): no matrix of order 2M is formed.  Returns false (nothing written)
// when the block does not qualify or Y is numerically rank deficient.
bool lowrank_block(const cgd_instance &in, int idx, int k, const std::vector<std::vector<double>> &rk,
                   HostInst &hi, std::vector<HostBlock> &out, bool want_hnorm, cgd_status &st) {
    st = CGD_OK;
    const int M = in.M, n2 = 2 * M;
    if (k == 0 && in.alpha)
        for (int q = 0; q < M; ++q)
            if (cx(in.alpha, q) != cplx(0, 0)) return false;
    const std::vector<int> ks{k};
    for (int i = 0; i < M; ++i)
        if (bin_of_row(in, i, M, ks, false) == CGD_KEEP) return false;
    std::vector<int> sq;
    for (int q = 0; q < M; ++q)
        if (rk[q][k] != 0.0) sq.push_back(q);
    const int r = 2 * (int)sq.size();
    if (r > kLowRankMax || 2 * r > n2) return false;
    const int rr = std::max(r, 1);
    HostBlock hb;
    hb.inst = idx;
    hb.blk = hi.nblocks;
    hb.nb = 0;
    hb.lowrank = rr;
    hb.lr.assign((size_t)(in.L + 1) * rr * rr, cplx(0, 0));
    if (r == 0) {  // vacuum in this internal mode: H = 0, factor 1
        for (int l = 0; l < in.L; ++l) {
            bool any = false;
            for (int i = 0; i < M; ++i) any |= bin_of_row(in, i, M, ks, false) == l;
            if (any) hi.marg[l].push_back(BinMarginal{});
        }
        hi.nblocks++;
        out.push_back(std::move(hb));
        return true;
    }
    CMat Y(n2, r), C(r, r);
    for (size_t a = 0; a < sq.size(); ++a) {
        const int q = sq[a];
        for (int i = 0; i < M; ++i) {
            const cplx t = cx(in.T, (size_t)i * M + q);
            Y(i, 2 * a) = t;
            Y(M + i, 2 * a + 1) = std::conj(t);
        }
        const double sh = std::sinh(rk[q][k]), ch = std::cosh(rk[q][k]);
        C(2 * a, 2 * a) = C(2 * a + 1, 2 * a + 1) = sh * sh;
        C(2 * a, 2 * a + 1) = C(2 * a + 1, 2 * a) = sh * ch;
    }
    // |Y_rows| for a set of rows (all, or one bin's): Gram^1/2 and, when asked, its inverse
    auto abs_y = [&](const std::vector<int> &rows, CMat &S, CMat *Sinv) -> bool {
        CMat Gm(r, r);
        for (int i : rows)
            for (int a = 0; a < r; ++a)
                for (int b = 0; b < r; ++b) Gm(a, b) += std::conj(Y(i, a)) * Y(i, b);
        std::vector<double> g;
        CMat U;
        if (!hermitian_eig_ql(Gm, g, U)) return false;
        double gmax = 0.0, gmin = INFINITY;
        for (double v : g) { gmax = std::max(gmax, v); gmin = std::min(gmin, v); }
        if (Sinv && !(gmin > 1e-12 * gmax)) return false;
        S = CMat(r, r);
        if (Sinv) *Sinv = CMat(r, r);
        for (int a = 0; a < r; ++a)
            for (int b = 0; b < r; ++b)
                for (int c2 = 0; c2 < r; ++c2) {
                    const cplx u = U(a, c2) * std::conj(U(b, c2));
                    S(a, b) += u * std::sqrt(std::max(g[c2], 0.0));
                    if (Sinv) (*Sinv)(a, b) += u / std::sqrt(g[c2]);
                }
        return true;
    };
    auto sandwich = [&](const CMat &S) {  // S C S
        CMat Z(r, r);
        for (int a = 0; a < r; ++a)
            for (int b = 0; b < r; ++b)
                for (int c1 = 0; c1 < r; ++c1)
                    for (int c2 = 0; c2 < r; ++c2) Z(a, b) += S(a, c1) * C(c1, c2) * S(c2, b);
        return Z;
    };
    std::vector<int> all(n2);
    for (int i = 0; i < n2; ++i) all[i] = i;
    CMat S, Sinv, W;
    if (!abs_y(all, S, &Sinv)) return false;
    std::vector<double> z;
    if (!hermitian_eig_ql(sandwich(S), z, W)) {
        st = fail(CGD_ERR_NUMERIC, "instance " + std::to_string(idx) + ": eigensolver");
        return true;
    }
    double ld = 0.0;
    std::vector<double> lam(r);
    for (int a = 0; a < r; ++a) {
        if (!(z[a] > -0.5)) {
            st = fail(CGD_ERR_NONPHYSICAL, "instance " + std::to_string(idx) + ": covariance violates Sigma > I/2");
            return true;
        }
        ld += std::log1p(z[a]);
        lam[a] = z[a] / (1.0 + z[a]);
        if (want_hnorm) hi.hnorm = std::max(hi.hnorm, std::fabs(lam[a]));
    }
    hi.logpr0 += -0.5 * ld;  // Eq. vacuum_probability, no displacement
    // marginal of every bin: a tridiagonal form of |Y_b| C |Y_b| (same nonzero spectrum)
    for (int l = 0; l < in.L; ++l) {
        std::vector<int> rows;
        for (int i = 0; i < n2; ++i)
            if (bin_of_row(in, i, M, ks, false) == l) rows.push_back(i);
        if (rows.empty()) continue;
        CMat Sb;
        if (!abs_y(rows, Sb, nullptr)) {
            st = fail(CGD_ERR_NUMERIC, "instance " + std::to_string(idx) + ": eigensolver");
            return true;
        }
        BinMarginal bm;
        hermitian_tridiag(sandwich(Sb), bm.d, bm.e, nullptr);
        hi.marg[l].push_back(std::move(bm));
    }
    // V = Y |Y|^-1 W, then G_g = diag(lambda) V^H E_g V
    CMat P(r, r);
    for (int a = 0; a < r; ++a)
        for (int b = 0; b < r; ++b)
            for (int c2 = 0; c2 < r; ++c2) P(a, b) += Sinv(a, c2) * W(c2, b);
    std::vector<cplx> v(r);
    for (int i = 0; i < n2; ++i) {
        for (int b = 0; b < r; ++b) {
            v[b] = cplx(0, 0);
            for (int a = 0; a < r; ++a) v[b] += Y(i, a) * P(a, b);
        }
        const int bn = bin_of_row(in, i, M, ks, false);
        const int g = bn < 0 ? 0 : bn + 1;
        for (int a = 0; a < r; ++a)
            for (int b = 0; b < r; ++b) hb.lr[((size_t)g * rr + a) * rr + b] += lam[a] * std::conj(v[a]) * v[b];
    }
    hi.nblocks++;
    out.push_back(std::move(hb));
    return true;
}

// Assemble one internal-mode block (all K modes when dense) of instance `in`:
// covariance matrix Sigma = I + [[N^T, M],[M^*, N]] (Sec. II), H = I - Sigma^-1,
// gamma = X Sigma^-1 zbar, the vacuum-probability term, unmeasured modes
// integrated out, and optionally the largest bin eliminated through its
// eigenbasis.
cgd_status assemble_block(const cgd_instance &in, int idx, const std::vector<int> &kset, bool dense,
                          bool use_schur, const std::vector<std::vector<double>> &rk, HostInst &hi,
                          std::vector<HostBlock> &out, std::vector<GradHost> *grads, bool want_hnorm,
                          bool lowrank_ok) {
    if (lowrank_ok && kset.size() == 1 && grads == nullptr) {
        cgd_status st = CGD_OK;
        if (lowrank_block(in, idx, kset[0], rk, hi, out, want_hnorm, st)) return st;
    }
    const int M = in.M;
    const int nk = (int)kset.size();
    const int m = M * nk;  // modes in this block
    const int n2 = 2 * m;
    // normally ordered moments: N = T^* diag(sinh^2) T^T, Mm = T diag(sinh cosh) T^T per internal mode
    CMat N(m, m), Mm(m, m);
    std::vector<cplx> beta(m, cplx(0, 0));
    std::vector<double> sh2(M), shch(M);
    for (int a = 0; a < nk; ++a) {
        const int k = kset[a];
        for (int q = 0; q < M; ++q) {
            const double sh = std::sinh(rk[q][k]), ch = std::cosh(rk[q][k]);
            sh2[q] = sh * sh;
            shch[q] = sh * ch;
        }
        for (int i = 0; i < M; ++i)
            for (int j = 0; j < M; ++j) {
                cplx sn(0, 0), sm(0, 0);
                for (int q = 0; q < M; ++q) {
                    const cplx tiq = cx(in.T, (size_t)i * M + q), tjq = cx(in.T, (size_t)j * M + q);
                    sn += std::conj(tiq) * tjq * sh2[q];
                    sm += tiq * tjq * shch[q];
                }
                const int ii = dense ? i * nk + a : i, jj = dense ? j * nk + a : j;
                N(ii, jj) = sn;
                Mm(ii, jj) = sm;
            }
        if (k == 0 && in.alpha)
            for (int i = 0; i < M; ++i) {
                cplx b(0, 0);
                for (int q = 0; q < M; ++q) b += cx(in.T, (size_t)i * M + q) * cx(in.alpha, q);
                beta[dense ? i * nk + a : i] = b;
            }
    }
    CMat Sig = CMat::eye(n2);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
            Sig(i, j) += N(j, i);
            Sig(i, m + j) += Mm(i, j);
            Sig(m + i, j) += std::conj(Mm(i, j));
            Sig(m + i, m + j) += N(i, j);
        }
    std::vector<cplx> zbar(n2);
    bool displaced = false;
    for (int i = 0; i < m; ++i) {
        zbar[i] = beta[i];
        zbar[m + i] = std::conj(beta[i]);
        if (beta[i] != cplx(0, 0)) displaced = true;
    }
    // marginal data of every bin for the tail bound (rows of both halves)
    for (int l = 0; l < in.L; ++l) {
        std::vector<int> idx;
        for (int i = 0; i < n2; ++i)
            if (bin_of_row(in, i, m, kset, dense) == l) idx.push_back(i);
        if (idx.empty()) continue;
        const int k = (int)idx.size();
        CMat R(k, k);
        for (int a = 0; a < k; ++a)
            for (int b = 0; b < k; ++b) R(a, b) = Sig(idx[a], idx[b]) - (a == b ? 1.0 : 0.0);
        BinMarginal bm;
        CMat Qd;
        hermitian_tridiag(R, bm.d, bm.e, displaced ? &Qd : nullptr);
        if (displaced) {
            bm.z.assign(k, cplx(0, 0));
            for (int a = 0; a < k; ++a)
                for (int b = 0; b < k; ++b) bm.z[a] += std::conj(Qd(b, a)) * zbar[idx[b]];
        }
        hi.marg[l].push_back(std::move(bm));
    }
    // uncertainty relation: Sigma - I/2 > 0  <=>  spec(H) inside (-1, 1)
    {
        CMat Sh = Sig;
        for (int i = 0; i < n2; ++i) Sh(i, i) -= 0.5;
        if (!hermitian_positive_definite(Sh))
            return fail(CGD_ERR_NONPHYSICAL, "instance " + std::to_string(idx) + ": covariance violates Sigma > I/2");
    }
    if (want_hnorm) {  // ||H||_2 = max_i |1 - 1/sigma_i| over the eigenvalues sigma_i of Sigma
        std::vector<double> sg;
        if (!hermitian_eigvals(Sig, sg)) return fail(CGD_ERR_NUMERIC, "instance " + std::to_string(idx) + ": eigensolver");
        for (double v : sg) hi.hnorm = std::max(hi.hnorm, std::fabs(1.0 - 1.0 / v));
    }
    CMat Sinv;
    if (!inverse(Sig, Sinv)) return fail(CGD_ERR_NUMERIC, "instance " + std::to_string(idx) + ": singular covariance");
    std::vector<cplx> v(n2, cplx(0, 0));  // Sigma^-1 zbar
    for (int i = 0; i < n2; ++i)
        for (int j = 0; j < n2; ++j) v[i] += Sinv(i, j) * zbar[j];
    cplx quad(0, 0);
    for (int i = 0; i < n2; ++i) quad += std::conj(zbar[i]) * v[i];
    const double ld = logdet_hpd(Sig);
    if (!std::isfinite(ld)) return fail(CGD_ERR_NUMERIC, "instance " + std::to_string(idx) + ": log det Sigma");
    hi.logpr0 += -0.5 * quad.real() - 0.5 * ld;  // Eq. vacuum_probability

    // Bordered H' over the state rows srow (every row that is not kept): H,
    // column -X gamma = -Sigma^-1 zbar, row -gamma^T (last).  Density mode: the
    // kept modes' rows krow (first half, then second half) come between them as
    // a border with columns -H_{srow, g}, rows -A_{g, srow} = -H_{X g, srow}, the
    // block A_GG = H_{X g, g'} and gamma_G = v_{X g} against the gamma border,
    // so that the Schur complement left after eliminating the state rows holds
    // the kept modes' quadratic form (see density_expand).
    auto xp = [m](int i) { return i < m ? i + m : i - m; };
    std::vector<int> srow, krow;
    {
        std::vector<int> kA;
        for (int i = 0; i < m; ++i)
            if (bin_of_row(in, i, m, kset, dense) == CGD_KEEP) kA.push_back(i);
        for (int i = 0; i < n2; ++i)
            if (bin_of_row(in, i, m, kset, dense) != CGD_KEEP) srow.push_back(i);
        for (int i : kA) krow.push_back(i);
        for (int i : kA) krow.push_back(i + m);
    }
    const int ns = (int)srow.size(), nkr = (int)krow.size();
    const int ig = ns + nkr;  // gamma border
    const int nf = ig + (displaced ? 1 : 0);
    CMat Hf(nf, nf);
    for (int a = 0; a < ns; ++a)
        for (int b = 0; b < ns; ++b) Hf(a, b) = (srow[a] == srow[b] ? 1.0 : 0.0) - Sinv(srow[a], srow[b]);
    for (int a = 0; a < ns; ++a)
        for (int q = 0; q < nkr; ++q) {
            Hf(a, ns + q) = Sinv(srow[a], krow[q]);
            Hf(ns + q, a) = Sinv(xp(krow[q]), srow[a]);
        }
    for (int q = 0; q < nkr; ++q)
        for (int q2 = 0; q2 < nkr; ++q2)
            Hf(ns + q, ns + q2) = (xp(krow[q]) == krow[q2] ? 1.0 : 0.0) - Sinv(xp(krow[q]), krow[q2]);
    std::vector<int32_t> rb(nf, -1);
    for (int a = 0; a < ns; ++a) rb[a] = bin_of_row(in, srow[a], m, kset, dense);
    if (displaced) {
        for (int a = 0; a < ns; ++a) {
            Hf(a, ig) = -v[srow[a]];      // X gamma = Sigma^-1 zbar
            Hf(ig, a) = -v[xp(srow[a])];  // gamma = X Sigma^-1 zbar
        }
        for (int q = 0; q < nkr; ++q) Hf(ns + q, ig) = Hf(ig, ns + q) = v[xp(krow[q])];
        Hf(ig, ig) = 0.0;
    }

    if (grads) {
        GradHost g;
        g.inst = idx;
        g.k = kset[0];
        g.n2 = n2;
        g.bordered = displaced ? 1 : 0;
        g.Sinv = Sinv;
        g.v = v;
        g.Hf = Hf;
        g.rb = rb;
        grads->push_back(std::move(g));
    }

    // integrate out unmeasured modes: det S = det(I - H_UU) det(I - D_R H_red),
    // H_red = H_RR + H_RU (I - H_UU)^-1 H_UR (the reduced Gaussian state)
    std::vector<int> U, R;
    for (int i = 0; i < ns; ++i) (rb[i] < 0 ? U : R).push_back(i);
    for (int i = ns; i < nf; ++i) R.push_back(i);  // borders last
    CMat Hr;
    std::vector<int32_t> rbr;
    if (!U.empty()) {
        const int nu = (int)U.size(), nr = (int)R.size();
        CMat Suu(nu, nu), Hur(nu, nr), Hru(nr, nu);
        for (int a = 0; a < nu; ++a) {
            for (int b = 0; b < nu; ++b) Suu(a, b) = (a == b ? 1.0 : 0.0) - Hf(U[a], U[b]);
            for (int b = 0; b < nr; ++b) Hur(a, b) = Hf(U[a], R[b]);
        }
        for (int a = 0; a < nr; ++a)
            for (int b = 0; b < nu; ++b) Hru(a, b) = Hf(R[a], U[b]);
        const double ldu = logdet_hpd(Suu);
        if (!std::isfinite(ldu)) return fail(CGD_ERR_NUMERIC, "instance " + std::to_string(idx) + ": reduction");
        hi.logpr0 += -0.5 * ldu;
        CMat X;
        if (!solve(Suu, Hur, X)) return fail(CGD_ERR_NUMERIC, "instance " + std::to_string(idx) + ": reduction solve");
        CMat corr = matmul(Hru, X);
        Hr = CMat(nr, nr);
        for (int a = 0; a < nr; ++a)
            for (int b = 0; b < nr; ++b) Hr(a, b) = Hf(R[a], R[b]) + corr(a, b);
        rbr.resize(nr);
        for (int a = 0; a < nr; ++a) rbr[a] = rb[R[a]];
    } else {
        Hr = Hf;
        rbr = rb;
    }
    const int nr = Hr.r;
    if (nr == 0) return CGD_OK;  // nothing measured, nothing displaced: constant factor only

    HostBlock hb;
    hb.inst = idx;
    hb.blk = hi.nblocks;
    hb.bordered = displaced ? 1 : 0;
    hb.nkeep = nkr;
    if (nkr) {
        // variable positions: (v_1..v_g, u_1..u_g); a first-half row is the ket
        // variable x of its mode (u), a second-half row the bra variable y (v)
        const std::vector<int> kf = kept_fine_modes(in);
        const int g = (int)kf.size();
        for (int q = 0; q < nkr; ++q) {
            const int md = krow[q] % m;
            const int fine = dense ? (md / nk) * in.K + kset[md % nk] : md * in.K + kset[0];
            const int kidx = (int)(std::lower_bound(kf.begin(), kf.end(), fine) - kf.begin());
            hb.kv.push_back(krow[q] < m ? g + kidx : kidx);
        }
    }
    // eliminate the bin with most rows through the eigenbasis of its (Hermitian) block
    int axis = -1;
    if (use_schur) {
        std::vector<int> cnt(in.L, 0);
        for (int a = 0; a < nr; ++a)
            if (rbr[a] >= 0) cnt[rbr[a]]++;
        int best = 0;
        for (int l = 0; l < in.L; ++l)
            if (cnt[l] > best) { best = cnt[l]; axis = l; }
    }
    if (axis >= 0) {
        std::vector<int> A, Bv;
        for (int a = 0; a < nr; ++a) (rbr[a] == axis ? A : Bv).push_back(a);  // border stays last in B
        const int na = (int)A.size(), nbB = (int)Bv.size();
        CMat Haa(na, na);
        for (int a = 0; a < na; ++a)
            for (int b = 0; b < na; ++b) Haa(a, b) = 0.5 * (Hr(A[a], A[b]) + std::conj(Hr(A[b], A[a])));
        CMat V;
        // with no rows left after the elimination (one bin) only the eigenvalues matter
        const bool ok = nbB == 0 ? hermitian_eigvals(Haa, hb.eig) : hermitian_eig_ql(Haa, hb.eig, V);
        if (!ok) return fail(CGD_ERR_NUMERIC, "instance " + std::to_string(idx) + ": eigensolver");
        for (double lam : hb.eig)
            if (!(std::fabs(lam) < 1.0)) return fail(CGD_ERR_NONPHYSICAL, "instance " + std::to_string(idx) + ": |eig(H)| >= 1");
        CMat Hba(nbB, na), Hab(na, nbB);
        hb.H = CMat(nbB, nbB);
        for (int a = 0; a < nbB; ++a) {
            for (int b = 0; b < na; ++b) Hba(a, b) = Hr(Bv[a], A[b]);
            for (int b = 0; b < nbB; ++b) hb.H(a, b) = Hr(Bv[a], Bv[b]);
        }
        for (int a = 0; a < na; ++a)
            for (int b = 0; b < nbB; ++b) Hab(a, b) = Hr(A[a], Bv[b]);
        if (nbB > 0) {
            hb.P = matmul(Hba, V);
            hb.Q = matmul(adjoint(V), Hab);
        }
        hb.schur_axis = axis;
        hb.nb = nbB;
        hb.rowbin.resize(nbB);
        for (int a = 0; a < nbB; ++a) hb.rowbin[a] = rbr[Bv[a]];
    } else {
        hb.H = Hr;
        hb.nb = nr;
        hb.rowbin = rbr;
    }
    out.push_back(std::move(hb));
    hi.nblocks++;
    return CGD_OK;
}

template <class T>
cgd_status upload(T **dptr, const std::vector<T> &host) {
    *dptr = nullptr;
    if (host.empty()) return CGD_OK;
    HIP_OK(hipMalloc((void **)dptr, sizeof(T) * host.size()));
    HIP_OK(hipMemcpy(*dptr, host.data(), sizeof(T) * host.size(), hipMemcpyHostToDevice));
    return CGD_OK;
}

constexpr int kG64 = kRegClasses + 1;

// timing slot of an LU launch: order buckets <=32, <=64, <=96, <=128, <=144, above
int lu_stage(int cls) { return cls < 5 ? CGD_STAGE_LU_REG0 + cls : CGD_STAGE_LU_BIG; }

struct LuClass {
    int cls = 0;  // class index within its group family
    std::vector<int32_t> jobs;
    std::vector<int64_t> prefix;
    int64_t nitems = 0;
    int32_t *d_jobs = nullptr;
    int64_t *d_prefix = nullptr;
    int32_t *d_hint = nullptr;  // per 64 items: the job of the first (LU range launches)
};

// Blocks that can take the Hessenberg route: the first bin eliminated through
// its eigenbasis, no displacement border, order within the reduction
// kernels' limit, and every row left in one other bin.  Returns that bin, or -1.
static int hess_bin(const HostBlock &h) {
    if (h.schur_axis < 0 || h.bordered || h.nkeep || h.nb < 1 || h.nb > hess_class_limit(kHessClasses - 1)) return -1;
    int hbin = -1;
    for (int32_t rb : h.rowbin) {
        if (rb < 0 || (hbin >= 0 && rb != hbin)) return -1;
        hbin = rb;
    }
    return hbin == h.schur_axis ? -1 : hbin;
}

// Blocks that can take the pair route: as above, but the rows left lie in two
// bins.  The bin with fewer values on the grid is eliminated per (w_A, w_P)
// pair by a partial LU (fewer pairs); the other must fit a reduction class.
constexpr int kPairMaxOrder = 480;
// The pair route is switched off: its kernels ended in a GPU memory fault on
// their first run and the cause is not found yet.
constexpr bool kPairRoute = false;
static bool pair_bins(const HostBlock &h, const InstDev &I, int &pbin, int &hbin) {
    if (!kPairRoute) return false;
    if (h.schur_axis < 0 || h.bordered || h.nkeep || h.nb < 2 || h.nb > kPairMaxOrder) return false;
    int b1 = -1, b2 = -1, n1 = 0, n2 = 0;
    for (int32_t rb : h.rowbin) {
        if (rb < 0 || rb == h.schur_axis) return false;
        if (b1 < 0 || rb == b1) {
            b1 = rb;
            ++n1;
        } else if (b2 < 0 || rb == b2) {
            b2 = rb;
            ++n2;
        } else {
            return false;
        }
    }
    if (b2 < 0) return false;
    auto nval = [&](int l) { return l == 0 ? I.H1 : I.G[l]; };
    const int lim = hess_class_limit(kHessClasses - 1);
    const bool first = nval(b1) <= nval(b2);
    pbin = first ? b1 : b2;
    hbin = first ? b2 : b1;
    if ((first ? n2 : n1) > lim) std::swap(pbin, hbin);
    return (pbin == b1 ? n2 : n1) <= lim;
}

// Hessenberg-route jobs of one size class: reduction (one workgroup per k_A)
// and factorisations (one workgroup per k_A and 16 values of k_B)
struct HessClass {
    std::vector<HessDev> jobs;
    std::vector<int64_t> rprefix, dprefix;
    int64_t rnwg = 0, dnwg = 0;
    HessDev *d_jobs = nullptr;
    int64_t *d_rprefix = nullptr, *d_dprefix = nullptr;
};

struct DftStage {
    std::vector<DftStageDev> desc;
    std::vector<int64_t> prefix;
    int64_t total = 0;
    DftStageDev *d_desc = nullptr;
    int64_t *d_prefix = nullptr;
    // descriptors with extent K <= kDftColsK (dft_cols: one thread per column)
    std::vector<DftStageDev> cdesc;
    std::vector<int64_t> cprefix;
    int64_t ctotal = 0;
    DftStageDev *d_cdesc = nullptr;
    int64_t *d_cprefix = nullptr;
};

}  // namespace

struct cgd_ctx {
    int n_inst = 0;
    cgd_precision prec = CGD_PREC_FP64;
    double tol = 0;
    uint32_t flags = 0;
    hipStream_t stream = nullptr;
    std::vector<InstDev> inst;
    std::vector<BlockDev> blocks;
    std::vector<SchurDev> schur;
    std::vector<int64_t> schur_prefix;
    int64_t schur_nwg = 0;
    int schur_maxA = 0;
    // FP64 groups: register classes 0..kRegClasses-1, blocked kernel kRegClasses;
    // mixed path: FP32 MFMA groups for the first pass
    LuClass g64[kG64];
    LuClass g32[kMfmaClasses];
    LuClass g64one;  // FP64 blocks of order <= 16 (one tile) outside density mode: lu_mfma_f64<1,1,1>
    // low-rank blocks, one list per rank (a kernel instance each): one job per
    // instance, (first, count) into blk; prefix / ntiles count tiles of 16
    // blocks x a run of points
    struct LowRankList {
        std::vector<int32_t> blk;
        std::vector<int2> jobs;
        std::vector<int64_t> prefix;
        int64_t ntiles = 0;
        int gstride = 1, wstride = 1;  // LDS entries per block / per point
        int32_t *d_blk = nullptr;
        int2 *d_jobs = nullptr;
        int64_t *d_prefix = nullptr;
    } lowrank[kLowRankMax];
    size_t lowrank_blocks = 0;
    int big_ldw = 0, big_nwg = 0;
    // Hessenberg route
    std::vector<char> is_hess;
    std::vector<double> tau_scale;   // per block: factor on the FP32 error model (1 unless the sample showed more)
    std::vector<HessDev> hess_all;
    std::vector<int64_t> hess_sprefix;
    int64_t hess_spts = 0, hess_ntab = 0, hess_nec = 0;
    HessClass hcls[kHessClasses];
    HessDev *d_hess_all = nullptr;
    // pair route: partial LU of each (w_A, w_P) pair before the reduction
    std::vector<PairDev> pairs;
    std::vector<int64_t> pair_prefix;
    int64_t npairs = 0, s_region = 0;  // pairs; size of the S region after the uploaded pool
    int64_t pool_host = 0;             // elements of the matrix pool written by the host
    int pair_ldw = 0, pair_nwg = 0;
    PairDev *d_pairs = nullptr;
    int64_t *d_pair_prefix = nullptr;
    int32_t *d_perm = nullptr;
    double2 *d_pair_work = nullptr;
    int64_t *d_hess_sprefix = nullptr;
    double2 *d_eigc = nullptr, *d_htable = nullptr;
    std::vector<DftStage> stages;
    std::map<int, int64_t> tw_of;      // grid extent G -> its twiddles in d_tw
    double2 *d_tw = nullptr;           // exp(-2 pi i m / G), m < G, for every G in use
    std::vector<int64_t> prob_offsets, inst_pt_prefix;
    int64_t nprobs = 0, npts = 0, ngrid = 0, ncontrib = 0;
    int64_t ntab = 0;                  // values per evaluation: sum_i points_i * E_i
    // density mode: instances with kept modes, prefix of their points and of
    // their output matrices (one per heralding pattern), trailing Schur complement pool
    std::vector<int32_t> dinst;
    std::vector<int64_t> dprefix, hprefix;
    int64_t dnpts = 0, htotal = 0, nmat = 0, ntpool = 0, dens_lds = 0;
    int32_t *d_dinst = nullptr;
    int64_t *d_dprefix = nullptr, *d_hprefix = nullptr;
    double2 *d_tpool = nullptr;
    // device
    InstDev *d_inst = nullptr;
    BlockDev *d_blocks = nullptr;
    SchurDev *d_schur = nullptr;
    int64_t *d_schur_prefix = nullptr;
    int64_t *d_inst_pt_prefix = nullptr;
    double2 *d_pool = nullptr;
    int32_t *d_rb = nullptr;
    double *d_eig = nullptr;
    double2 *d_contrib = nullptr, *d_logg = nullptr, *d_gA = nullptr, *d_gB = nullptr, *d_work = nullptr;
    // mixed path
    float2 *d_pool32 = nullptr;
    double2 *d_logg32 = nullptr;
    int64_t list_cap[kG64] = {};
    int64_t list_off[kG64] = {};       // first entry of each FP64 class's list in d_list (-1: none)
    int64_t list_total = 0;
    int2 *d_list = nullptr;
    int64_t *d_list_off = nullptr;
    int *d_counts = nullptr;
    unsigned long long *d_hist = nullptr;  // per instance: bucket sums of c_k |G_k| (fixed point)
    int *d_cut = nullptr;              // per instance: buckets up to cut are factorised again in FP64
    int *d_status = nullptr;
    int *h_status = nullptr;
    hipEvent_t ev_status = nullptr;
    bool status_pending = false;
    bool poisoned = false;
    // gradient
    std::vector<GradHost> grads;
    std::vector<HostInstCopy> hinst_copy;
    std::vector<GradBlockDev> gblocks;
    LuClass gadj[kAdjClasses];
    int adj_chunk = 16;
    int64_t part_stride = 0, adj_items = 0, z_total = 0, adj_total = 0;
    std::vector<int64_t> z_elem_prefix, adj_off;
    std::vector<DftStage> adj_stages;
    GradBlockDev *d_gblocks = nullptr;
    double2 *d_gpool = nullptr, *d_partial = nullptr, *d_z = nullptr, *d_adjA = nullptr, *d_adjB = nullptr,
            *d_ghat = nullptr;
    double2 *d_adj_work = nullptr;  // adjoint class 3: adj_nwg workspaces of adj_ldw x adj_ldw
    int adj_ldw = 0, adj_nwg = 0;
    int32_t *d_grb = nullptr;
    int64_t *d_z_prefix = nullptr, *d_adj_off = nullptr, *d_prob_prefix = nullptr;
    // HIP graph of the evaluation
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t gexec = nullptr;
    double *g_probs = nullptr, *g_err = nullptr;
    bool evaluated = false;
    bool last_static = false;          // the last evaluation was cgd_eval_static
    int reg_var[kRegClasses] = {};     // autotuner: thread grid of the FP64 register kernel per class
    int mfma_var[kMfmaClasses] = {};   // autotuner: wave layout of the FP32 MFMA kernel per class
    std::string tune_json;             // autotuner report
    std::vector<double> wrap_bound;    // per instance: sum_l bound on Pr(b_l >= G_l)
    std::vector<int32_t> grid_used;    // grid extents of every instance (auto entries resolved)
    int device = -1;                   // device current at cgd_create
    bool timing = false;
    // per-launch timing: event pairs recorded around each launch of a stage (eager
    // evaluations with timing on); a stage's time is the sum over its launches
    std::vector<hipEvent_t> tev;       // pool, two per pair
    std::vector<int> tev_stage;        // stage of each recorded pair
    size_t tev_open = 0;
    bool stage_ran[CGD_NSTAGES] = {};
    double work_flops[CGD_NSTAGES] = {}, work_bytes[CGD_NSTAGES] = {};
};

namespace {

void free_ctx(cgd_ctx *c) {
    if (!c) return;
    auto fr = [](void *p) { if (p) (void)hipFree(p); };
    fr(c->d_inst); fr(c->d_blocks); fr(c->d_schur); fr(c->d_schur_prefix); fr(c->d_inst_pt_prefix);
    fr(c->d_pool); fr(c->d_rb); fr(c->d_eig); fr(c->d_contrib); fr(c->d_logg); fr(c->d_gA); fr(c->d_gB);
    fr(c->d_tpool); fr(c->d_dinst); fr(c->d_dprefix); fr(c->d_hprefix);
    fr(c->d_work); fr(c->d_status); fr(c->d_pool32); fr(c->d_logg32); fr(c->d_list); fr(c->d_list_off);
    fr(c->d_counts); fr(c->d_hist); fr(c->d_cut);
    for (auto &k : c->g64) { fr(k.d_jobs); fr(k.d_prefix); fr(k.d_hint); }
    fr(c->g64one.d_jobs); fr(c->g64one.d_prefix); fr(c->g64one.d_hint);
    for (auto &lr : c->lowrank) { fr(lr.d_blk); fr(lr.d_jobs); fr(lr.d_prefix); }
    for (auto &k : c->g32) { fr(k.d_jobs); fr(k.d_prefix); fr(k.d_hint); }
    for (auto &s : c->stages) { fr(s.d_desc); fr(s.d_prefix); fr(s.d_cdesc); fr(s.d_cprefix); }
    fr(c->d_tw);
    for (auto &s : c->adj_stages) { fr(s.d_desc); fr(s.d_prefix); }
    for (auto &h : c->hcls) { fr(h.d_jobs); fr(h.d_rprefix); fr(h.d_dprefix); }
    fr(c->d_hess_all); fr(c->d_hess_sprefix); fr(c->d_eigc); fr(c->d_htable);
    fr(c->d_pairs); fr(c->d_pair_prefix); fr(c->d_perm); fr(c->d_pair_work);
    for (auto &k : c->gadj) { fr(k.d_jobs); fr(k.d_prefix); }
    fr(c->d_adj_work);
    fr(c->d_gblocks); fr(c->d_gpool); fr(c->d_partial); fr(c->d_z); fr(c->d_adjA); fr(c->d_adjB); fr(c->d_ghat);
    fr(c->d_grb); fr(c->d_z_prefix); fr(c->d_adj_off); fr(c->d_prob_prefix);
    for (hipEvent_t e : c->tev) (void)hipEventDestroy(e);
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->h_status) (void)hipHostFree(c->h_status);
    if (c->ev_status) (void)hipEventDestroy(c->ev_status);
    delete c;
}

// Route for the blocks hess_bin or pair_bins accepts (all of them, or none),
// unless a flag forces it: the Hessenberg route replaces a factorisation per
// point by one reduction per value of w_A (pair route: per (w_A, w_P) pair,
// after a partial LU) plus an O(n^2) factorisation per point.  The reductions
// run one per compute unit and are latency bound, so with few values of w_A,
// or few points per reduction, the factorisations per point are faster.  Both
// sides are estimated from per-kernel times measured on MI355X, in
// microseconds of one compute unit:
//   reduction    (n - 2) steps of t_step (1.4, 2.0, 3.0, 3.4 us for orders
//                <= 32, 64, 96, 144), one reduction per compute unit at a time;
//   Hessenberg   3.7 (n / 144)^2 per point;
//   partial LU   680 (n^3 - nB^3) / 192^3 per pair (blocked FP64 LU);
//   LU per point orders <= 144: 148 (n / 144)^3 (FP64), 70 (n / 144)^3
//                (mixed, including the share factorised again in FP64);
//                above: 680 (n / 192)^3 (FP64), 130 (n / 192)^3 (mixed).
bool choose_hessenberg(const cgd_ctx *c, const std::vector<HostBlock> &hb, std::vector<int> &hbins,
                       std::vector<int> &pbins) {
    bool any = false;
    for (size_t b = 0; b < hb.size(); ++b) {
        pbins[b] = -1;
        if (hb[b].lowrank) {  // no factorisation to replace
            hbins[b] = -1;
            continue;
        }
        hbins[b] = hess_bin(hb[b]);
        if (hbins[b] < 0 && !pair_bins(hb[b], c->inst[hb[b].inst], pbins[b], hbins[b])) {
            hbins[b] = -1;
            pbins[b] = -1;
        }
        any |= hbins[b] >= 0;
    }
    if (!any || (c->flags & CGD_FLAG_NO_HESSENBERG)) return false;
    if (c->flags & CGD_FLAG_HESSENBERG) return true;
    int ncu = 0, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0)
        ncu = 256;
    static constexpr double t_step[kHessClasses] = {1.4, 2.0, 3.0, 3.4};
    double red_n[kHessClasses] = {};  // total reductions per class
    double red_t[kHessClasses] = {};  // longest reduction per class
    double det_cu = 0.0, plu_cu = 0.0, lu_cu = 0.0;
    const bool mixed = c->prec == CGD_PREC_MIXED;
    for (size_t b = 0; b < hb.size(); ++b) {
        if (hbins[b] < 0) continue;
        const HostBlock &h = hb[b];
        const InstDev &I = c->inst[h.inst];
        auto nval = [&](int l) { return (double)(l == 0 ? I.H1 : I.G[l]); };
        double nred = nval(h.schur_axis);
        int nH = h.nb;
        if (pbins[b] >= 0) {
            nH = 0;
            for (int32_t rb : h.rowbin) nH += rb == hbins[b];
            nred *= nval(pbins[b]);
            const double n3 = (double)h.nb * h.nb * h.nb, h3 = (double)nH * nH * nH;
            plu_cu += nred * 680.0 * (n3 - h3) / (192.0 * 192.0 * 192.0);
        }
        int cls = 0;
        while (nH > hess_class_limit(cls)) ++cls;
        const double r = nH / 144.0;
        red_n[cls] += nred;
        red_t[cls] = std::max(red_t[cls], (nH - 2) * t_step[cls]);
        det_cu += nred * nval(hbins[b]) * 3.7 * r * r;
        const double q = h.nb <= 144 ? h.nb / 144.0 : h.nb / 192.0;
        const double per = h.nb <= 144 ? (mixed ? 70.0 : 148.0) : (mixed ? 130.0 : 680.0);
        lu_cu += (double)I.npts * per * q * q * q;
    }
    double t_hess = (det_cu + plu_cu) / ncu;
    for (int k = 0; k < kHessClasses; ++k) t_hess += std::ceil(red_n[k] / ncu) * red_t[k];
    return t_hess < lu_cu / ncu;
}

cgd_status check_status(cgd_ctx *c) {
    if (c->poisoned) return fail(CGD_ERR_NUMERIC, "a previous evaluation hit a pivot outside the right half-plane");
    if (c->status_pending) {
        if (hipEventQuery(c->ev_status) == hipSuccess) {
            c->status_pending = false;
            if (*c->h_status) {
                c->poisoned = true;
                return fail(CGD_ERR_NUMERIC, "a previous evaluation hit a pivot outside the right half-plane");
            }
        }
    }
    return CGD_OK;
}

// Device structures of the adjoint: full bordered block matrices, work lists
// (chunks of grid points), partial and reduced sums, adjoint-DFT passes.
cgd_status build_grad(cgd_ctx *c, int n_inst) {
    std::vector<double2> gpool;
    std::vector<int32_t> grb;
    for (int k = 0; k < kAdjClasses; ++k) c->gadj[k].cls = k;
    c->gblocks.resize(c->grads.size());
    std::vector<int> bcls(c->grads.size());
    int64_t zoff = 0;
    for (size_t b = 0; b < c->grads.size(); ++b) {
        const GradHost &g = c->grads[b];
        GradBlockDev &d = c->gblocks[b];
        std::memset(&d, 0, sizeof(d));
        d.inst = g.inst;
        d.nb = g.Hf.r;
        d.bordered = g.bordered;
        int cls = -1;
        for (int k = 0; k < kAdjClasses; ++k)
            if (d.nb <= adj_class_limit(k)) { cls = k; break; }
        if (cls < 0)
            return fail(CGD_ERR_ARG, "CGD_FLAG_GRAD: block order above " + std::to_string(kAdjBigMax) +
                                         " is not supported");
        bcls[b] = cls;
        d.h_off = (int64_t)gpool.size();
        for (const cplx &z : g.Hf.a) gpool.push_back(make_double2(z.real(), z.imag()));
        d.rb_off = (int64_t)grb.size();
        grb.insert(grb.end(), g.rb.begin(), g.rb.end());
        const int64_t np = c->inst[g.inst].npts;
        d.nchunks = (int32_t)((np + c->adj_chunk - 1) / c->adj_chunk);
        const int n = d.nb - d.bordered;
        d.z_off = zoff;
        c->z_elem_prefix.push_back(zoff);
        zoff += (int64_t)n * n + n + 1;
        c->part_stride = std::max<int64_t>(c->part_stride, (int64_t)n * n + n + 1);
    }
    // work items (chunks of grid points) numbered class by class, so that each
    // class launch covers one contiguous range
    int64_t item = 0;
    for (int k = 0; k < kAdjClasses; ++k)
        for (size_t b = 0; b < c->grads.size(); ++b) {
            if (bcls[b] != k) continue;
            GradBlockDev &d = c->gblocks[b];
            d.first_item = item;
            c->gadj[k].jobs.push_back((int32_t)b);
            c->gadj[k].prefix.push_back(item);
            item += d.nchunks;
        }
    c->adj_items = item;
    c->z_total = zoff;
    // adjoint DFT passes: axis 0 first, (N_l + 1) -> H1 (axis 0) or G_l
    c->adj_off.assign(n_inst, 0);
    int64_t off = 0;
    int Lmax = 0;
    for (int i = 0; i < n_inst; ++i) {
        c->adj_off[i] = off;
        off += std::max(c->inst[i].npts, c->inst[i].nprobs);
        Lmax = std::max(Lmax, c->inst[i].L);
    }
    c->adj_total = off;
    c->adj_stages.resize(Lmax);
    for (int s2 = 0; s2 < Lmax; ++s2) {
        DftStage &st = c->adj_stages[s2];
        for (int i = 0; i < n_inst; ++i) {
            const InstDev &I = c->inst[i];
            if (I.L <= s2) continue;
            const int a = s2;
            int64_t dims[kMaxBins];
            for (int l = 0; l < I.L; ++l) dims[l] = l < a ? (l == 0 ? I.H1 : I.G[l]) : (I.N[l] + 1);
            DftStageDev d;
            std::memset(&d, 0, sizeof(d));
            d.inst = i;
            d.K = I.N[a] + 1;
            d.Bout = a == 0 ? I.H1 : I.G[a];
            d.G = I.G[a];
            d.tw_off = c->tw_of.at(d.G);
            d.final_stage = 0;
            d.outer = 1;
            for (int l = 0; l < a; ++l) d.outer *= dims[l];
            d.inner = 1;
            for (int l = a + 1; l < I.L; ++l) d.inner *= dims[l];
            d.in_off = c->adj_off[i];
            d.out_off = c->adj_off[i];
            d.scale = 1.0;
            st.prefix.push_back(st.total);
            st.total += d.outer * d.Bout * d.inner;
            st.desc.push_back(d);
        }
    }
    cgd_status s;
    if ((s = upload(&c->d_gblocks, c->gblocks)) != CGD_OK) return s;
    if ((s = upload(&c->d_gpool, gpool)) != CGD_OK) return s;
    if ((s = upload(&c->d_grb, grb)) != CGD_OK) return s;
    if ((s = upload(&c->d_z_prefix, c->z_elem_prefix)) != CGD_OK) return s;
    if ((s = upload(&c->d_adj_off, c->adj_off)) != CGD_OK) return s;
    std::vector<int64_t> pp(c->prob_offsets.begin(), c->prob_offsets.begin() + n_inst);
    if ((s = upload(&c->d_prob_prefix, pp)) != CGD_OK) return s;
    for (auto &k : c->gadj) {
        if ((s = upload(&k.d_jobs, k.jobs)) != CGD_OK) return s;
        if ((s = upload(&k.d_prefix, k.prefix)) != CGD_OK) return s;
    }
    for (auto &st : c->adj_stages) {
        if ((s = upload(&st.d_desc, st.desc)) != CGD_OK) return s;
        if ((s = upload(&st.d_prefix, st.prefix)) != CGD_OK) return s;
    }
    // class 3 (orders above the register kernels): a persistent grid, one
    // ldw x ldw workspace per workgroup
    {
        int64_t items3 = 0;
        c->adj_ldw = 0;
        for (int32_t b : c->gadj[3].jobs) {
            items3 += c->gblocks[b].nchunks;
            c->adj_ldw = std::max(c->adj_ldw, c->gblocks[b].nb);
        }
        c->adj_nwg = (int)std::min<int64_t>(items3, 512);
        if (c->adj_nwg > 0) {
            HIP_OK(prepare_adj_big(c->adj_ldw));
            HIP_OK(hipMalloc((void **)&c->d_adj_work,
                             sizeof(double2) * (size_t)c->adj_nwg * c->adj_ldw * c->adj_ldw));
        }
    }
    HIP_OK(hipMalloc((void **)&c->d_partial, sizeof(double2) * std::max<int64_t>(1, c->adj_items * c->part_stride)));
    HIP_OK(hipMalloc((void **)&c->d_z, sizeof(double2) * std::max<int64_t>(1, c->z_total)));
    HIP_OK(hipMalloc((void **)&c->d_adjA, sizeof(double2) * std::max<int64_t>(1, c->adj_total)));
    HIP_OK(hipMalloc((void **)&c->d_adjB, sizeof(double2) * std::max<int64_t>(1, c->adj_total)));
    HIP_OK(hipMalloc((void **)&c->d_ghat, sizeof(double2) * std::max<int64_t>(1, c->npts)));
    return CGD_OK;
}

// Chain rule, host FP64: from dL = Re[tr(Z_H dH) + Z_g^T dgamma + Z_0 dlogPr0]
// per internal block (H = I - Sigma^-1, gamma = X Sigma^-1 zbar,
// logPr0 = -1/2 zbar^H Sigma^-1 zbar - 1/2 log det Sigma) to the inputs.  For
// a complex input z with dL = Re(a dz + b conj(dz)) the reported gradient is
// dL/dRe z + i dL/dIm z = conj(a) + b.
// Contribution of internal block b to dL/dr (M), dL/dT (M*M) and dL/dalpha (M)
// of its instance, written to gr, gT, ga (zero-initialised by the caller).
void chain_rule_block(const cgd_ctx *c, size_t b, const std::vector<cplx> &zhost, std::vector<double> &gr,
                      std::vector<cplx> &gT, std::vector<cplx> &ga, std::vector<double> &gs) {
    const int64_t to = 0, ro = 0;
    {
        const GradHost &g = c->grads[b];
        const GradBlockDev &d = c->gblocks[b];
        const HostInstCopy &hc = c->hinst_copy[g.inst];
        const int M = hc.M, n = g.n2;
        const cplx *z = &zhost[d.z_off];
        CMat ZH(n, n);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) ZH(i, j) = z[(int64_t)i * n + j];
        std::vector<cplx> Zg(z + (int64_t)n * n, z + (int64_t)n * n + n);
        const cplx Z0 = z[(int64_t)n * n + n];
        const CMat &Si = g.Sinv;
        // Gamma = Si ZH Si - v (Zg^T X Si) + Z0 (v v^H - Si) / 2
        CMat Gm = matmul(matmul(Si, ZH), Si);
        std::vector<cplx> xz(n);  // X Zg
        for (int i = 0; i < n; ++i) xz[i] = Zg[i < M ? i + M : i - M];
        std::vector<cplx> rho(n, cplx(0, 0));  // rho^T = Zg^T X Si  ->  rho = Si^T X Zg
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) rho[j] += xz[i] * Si(i, j);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                Gm(i, j) += -g.v[i] * rho[j] + 0.5 * Z0 * (g.v[i] * std::conj(g.v[j]) - Si(i, j));
        // blocks of Gamma: dL = Re[tr(PhiN dN) + tr(G21 dM) + tr(G12 dM*)]
        CMat PhiN(M, M), G21(M, M), G12(M, M);
        for (int i = 0; i < M; ++i)
            for (int j = 0; j < M; ++j) {
                PhiN(i, j) = Gm(j, i) + Gm(M + i, M + j);
                G21(i, j) = Gm(M + i, j);
                G12(i, j) = Gm(i, M + j);
            }
        // T and internal-mode squeezing of this block
        CMat T(M, M);
        for (int i = 0; i < M; ++i)
            for (int j = 0; j < M; ++j) T(i, j) = hc.T[(size_t)i * M + j];
        const CMat Tt = transpose(T), Th = adjoint(T), Tc = conj(T);
        std::vector<double> nn(M), mm(M), dn(M), dm(M), drk(M);
        for (int j = 0; j < M; ++j) {
            const double r = hc.rk[j][g.k];
            nn[j] = std::sinh(r) * std::sinh(r);
            mm[j] = std::sinh(r) * std::cosh(r);
            dn[j] = std::sinh(2 * r);
            dm[j] = std::cosh(2 * r);
            const double ratio = hc.K == 1 ? 1.0 : hc.schmidt[g.k] / hc.schmidt[0];
            const double sq = std::sqrt(ratio), th = std::tanh(hc.r[j]);
            drk[j] = sq * (1.0 - th * th) / (1.0 - ratio * th * th);
        }
        auto diagl = [&](const std::vector<double> &w, const CMat &A) {  // diag(w) A
            CMat R = A;
            for (int i = 0; i < A.r; ++i)
                for (int j = 0; j < A.c; ++j) R(i, j) *= w[i];
            return R;
        };
        // coefficient of dT (tr(Xa dT)) and of dT* (tr(Xb dT*))
        CMat Xa = diagl(nn, matmul(Th, transpose(PhiN)));
        CMat t3 = diagl(mm, matmul(Tt, G21)), t4 = diagl(mm, matmul(Tt, transpose(G21)));
        CMat Xb = diagl(nn, matmul(Tt, PhiN));
        CMat t5 = diagl(mm, matmul(Th, G12)), t6 = diagl(mm, matmul(Th, transpose(G12)));
        for (size_t e = 0; e < Xa.a.size(); ++e) {
            Xa.a[e] += t3.a[e] + t4.a[e];
            Xb.a[e] += t5.a[e] + t6.a[e];
        }
        CMat Cn = matmul(matmul(Tt, PhiN), Tc), Cm1 = matmul(matmul(Tt, G21), T), Cm2 = matmul(matmul(Th, G12), Tc);
        for (int i = 0; i < M; ++i)
            for (int j = 0; j < M; ++j) gT[to + (size_t)i * M + j] += std::conj(Xa(j, i)) + Xb(j, i);
        // dL/dr_jk, then through r_jk = artanh(x), x = sqrt(lambda_k / lambda_0) tanh r_j,
        // to r_j and (k > 0) to lambda_k and lambda_0, each weight a free variable
        for (int j = 0; j < M; ++j) {
            const double dl = Cn(j, j).real() * dn[j] + (Cm1(j, j) + Cm2(j, j)).real() * dm[j];
            gr[ro + j] += dl * drk[j];
            if (hc.K > 1 && g.k > 0) {
                const double x = std::sqrt(hc.schmidt[g.k] / hc.schmidt[0]) * std::tanh(hc.r[j]);
                const double f = dl * x / (2.0 * (1.0 - x * x));  // dL/dr_jk * d r_jk / d log(lambda_k / lambda_0)
                gs[g.k] += f / hc.schmidt[g.k];
                gs[0] -= f / hc.schmidt[0];
            }
        }
        // displacement: zbar = (beta, beta*), beta = T alpha on internal mode 0
        if (g.k == 0 && hc.alpha) {
            std::vector<cplx> ab(M), bb(M);
            for (int i = 0; i < M; ++i) {
                ab[i] = rho[i] - 0.5 * Z0 * (std::conj(g.v[i]) + g.v[M + i]);
                bb[i] = rho[M + i] - 0.5 * Z0 * (std::conj(g.v[M + i]) + g.v[i]);
            }
            for (int i = 0; i < M; ++i)
                for (int j = 0; j < M; ++j) {
                    const cplx al = hc.alpha[j];
                    gT[to + (size_t)i * M + j] += std::conj(ab[i] * al) + bb[i] * std::conj(al);
                }
            for (int j = 0; j < M; ++j) {
                cplx aa(0, 0), bs(0, 0);
                for (int i = 0; i < M; ++i) {
                    aa += T(i, j) * ab[i];            // (T^T a_beta)_j
                    bs += std::conj(T(i, j)) * bb[i]; // (T^H b_beta)_j
                }
                ga[ro + j] += std::conj(aa) + bs;
            }
        }
    }
}

// Chain rule over all blocks on up to 16 host threads; each block writes its own
// buffers and the sums into gr, gT, ga are taken in block order (reproducible).
void chain_rule(const cgd_ctx *c, const std::vector<cplx> &zhost, std::vector<double> &gr, std::vector<cplx> &gT,
                std::vector<cplx> &ga, std::vector<double> &gs, const std::vector<int64_t> &roff,
                const std::vector<int64_t> &toff, const std::vector<int64_t> &soff) {
    const size_t nb = c->grads.size();
    std::vector<std::vector<double>> bgr(nb), bgs(nb);
    std::vector<std::vector<cplx>> bgT(nb), bga(nb);
    std::atomic<size_t> next{0};
    auto work = [&]() {
        for (size_t b; (b = next.fetch_add(1)) < nb;) {
            const int M = c->hinst_copy[c->grads[b].inst].M;
            bgr[b].assign(M, 0.0);
            bgT[b].assign((size_t)M * M, cplx(0, 0));
            bga[b].assign(M, cplx(0, 0));
            bgs[b].assign(c->hinst_copy[c->grads[b].inst].K, 0.0);
            chain_rule_block(c, b, zhost, bgr[b], bgT[b], bga[b], bgs[b]);
        }
    };
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const size_t nthr = std::min<size_t>({(size_t)16, (size_t)hw, nb});
    std::vector<std::thread> pool;
    for (size_t t = 1; t < nthr; ++t) pool.emplace_back(work);
    work();
    for (auto &t : pool) t.join();
    for (size_t b = 0; b < nb; ++b) {
        const int inst = c->grads[b].inst;
        for (size_t j = 0; j < bgr[b].size(); ++j) {
            gr[roff[inst] + j] += bgr[b][j];
            ga[roff[inst] + j] += bga[b][j];
        }
        for (size_t e = 0; e < bgT[b].size(); ++e) gT[toff[inst] + e] += bgT[b][e];
        for (size_t k = 0; k < bgs[b].size(); ++k) gs[soff[inst] + k] += bgs[b][k];
    }
}


// FP32 MFMA class of an order
int mfma_class_of(int nb) {
    int k = 0;
    while (nb > mfma_class_limit(k)) ++k;
    return k;
}

// LU work lists from the block descriptors: FP64 groups (everything on the
// FP64 path; on the mixed path the blocks without an FP32 pass), FP32 MFMA
// groups (mixed first pass) and the capacity of the mixed second-pass lists
// per FP64 group.
cgd_status make_lu_lists(cgd_ctx *c) {
    for (int k = 0; k < kG64; ++k) {
        LuClass &g = c->g64[k];
        g.cls = k;
        g.jobs.clear();
        g.prefix.clear();
        g.nitems = 0;
        c->list_cap[k] = 0;
    }
    for (int k = 0; k < kMfmaClasses; ++k) {
        LuClass &g = c->g32[k];
        g.cls = k;
        g.jobs.clear();
        g.prefix.clear();
        g.nitems = 0;
    }
    c->g64one.cls = 0;
    c->g64one.jobs.clear();
    c->g64one.prefix.clear();
    c->g64one.nitems = 0;
    for (size_t b = 0; b < c->blocks.size(); ++b) {
        const BlockDev &d = c->blocks[b];
        if (c->is_hess[b] || d.lowrank) continue;
        if (d.cls == kRegClasses) {
            if (d.nb > 480) return fail(CGD_ERR_ARG, "matrix order above 480 per block is not supported");
            c->big_ldw = std::max(c->big_ldw, d.nb);
        }
        const int64_t np = c->inst[d.inst].npts;
        LuClass *lc = &c->g64[d.cls];
        if (d.fp32) {
            lc = &c->g32[mfma_class_of(d.nb)];
            c->list_cap[d.cls] += np;
        } else if (d.nb <= 16 && !d.nkeep) {
            // one 16 x 16 tile: a kernel sized for it (a quarter of the
            // registers and no panels, so several times the waves per CU)
            lc = &c->g64one;
        }
        lc->prefix.push_back(lc->nitems);
        lc->jobs.push_back((int32_t)b);
        lc->nitems += np;
    }
    const int64_t big_items = c->g64[kRegClasses].nitems + c->list_cap[kRegClasses];
    if (big_items > 0) c->big_nwg = (int)std::min<int64_t>(big_items, 1024);
    return CGD_OK;
}

double lu_flops(double n) {
    double f = 0;
    for (int m = 0; m < (int)n; ++m) f += 8.0 * m * m + 6.0 * m;
    return f;
}

// flops of one block's factorisation: a density-mode block stops after the
// pivots of S, the border rows (m < nb - nS) are updated but not eliminated
double block_flops(const BlockDev &d) {
    if (!d.nkeep) return lu_flops(d.nb);
    const int nS = d.nb - d.nkeep - d.bordered;
    double f = 0;
    for (int m = d.nb - 1; m >= d.nb - nS; --m) f += 8.0 * m * m + 6.0 * m;
    return f;
}

// algorithmic flops of the LU stages per evaluation (FP32 first pass and
// FP64 groups; the re-factorised share of the mixed path is not counted)
void lu_work(cgd_ctx *c) {
    for (int k = 0; k < kG64; ++k) c->work_flops[lu_stage(k)] = 0.0;
    for (int k = 0; k < kG64; ++k)
        for (int32_t bj : c->g64[k].jobs) {
            const BlockDev &d = c->blocks[bj];
            c->work_flops[lu_stage(k)] += block_flops(d) * c->inst[d.inst].npts;
        }
    for (int k = 0; k < kMfmaClasses; ++k)
        for (int32_t bj : c->g32[k].jobs) {
            const BlockDev &d = c->blocks[bj];
            c->work_flops[lu_stage(k)] += lu_flops(d.nb) * c->inst[d.inst].npts;
        }
    for (int32_t bj : c->g64one.jobs) {
        const BlockDev &d = c->blocks[bj];
        c->work_flops[lu_stage(0)] += block_flops(d) * c->inst[d.inst].npts;
    }
}

// device copies of the work lists and the mixed path's list layout
cgd_status upload_lu_lists(cgd_ctx *c) {
    auto fr = [](void *p) { if (p) (void)hipFree(p); };
    cgd_status s;
    for (auto *grp : {&c->g64[0], &c->g32[0], &c->g64one}) {
        const int n = grp == &c->g64[0] ? kG64 : grp == &c->g32[0] ? kMfmaClasses : 1;
        for (int k = 0; k < n; ++k) {
            fr(grp[k].d_jobs);
            fr(grp[k].d_prefix);
            fr(grp[k].d_hint);
            grp[k].d_jobs = nullptr;
            grp[k].d_prefix = nullptr;
            grp[k].d_hint = nullptr;
            if ((s = upload(&grp[k].d_jobs, grp[k].jobs)) != CGD_OK) return s;
            if ((s = upload(&grp[k].d_prefix, grp[k].prefix)) != CGD_OK) return s;
            // the job of items 0, 64, 128, ...: the kernels start their job
            // lookup there instead of a binary search over the whole prefix
            const LuClass &g = grp[k];
            std::vector<int32_t> hint((size_t)((g.nitems + 63) / 64));
            int32_t j = 0;
            for (size_t q = 0; q < hint.size(); ++q) {
                const int64_t t = (int64_t)q * 64;
                while (j + 1 < (int32_t)g.prefix.size() && g.prefix[j + 1] <= t) ++j;
                hint[q] = j;
            }
            if (!hint.empty() && (s = upload(&grp[k].d_hint, hint)) != CGD_OK) return s;
        }
    }
    if (c->prec != CGD_PREC_MIXED) return CGD_OK;
    std::vector<int64_t> offs(kG64, -1);
    c->list_total = 0;
    for (int k = 0; k < kG64; ++k)
        if (c->list_cap[k] > 0) {
            offs[k] = c->list_off[k] = c->list_total;
            c->list_total += c->list_cap[k];
        } else {
            c->list_off[k] = -1;
        }
    fr(c->d_list);
    fr(c->d_list_off);
    c->d_list = nullptr;
    c->d_list_off = nullptr;
    HIP_OK(hipMalloc((void **)&c->d_list, sizeof(int2) * std::max<int64_t>(1, c->list_total)));
    return upload(&c->d_list_off, offs);
}

// Autotuner.  For every size class of per-point factorisations in this
// context, time each candidate kernel shape on a sample of the class's own
// (block, grid point) items spread evenly over its blocks (after building the
// Schur matrices, so that the inputs are the real ones): the thread grids of
// the FP64 register kernel and, on the mixed path, the wave layouts of the
// FP32 MFMA kernel.  The fastest shape of each kind is kept.  A mixed class
// whose best FP32 pass is not clearly faster than its best FP64 kernel (below
// kMixedFp32Gain of the FP64 time) runs directly in FP64: besides its own
// points that the budget sends back to FP64, an FP32 block raises the error
// bound of every point it belongs to and so the re-factorisation of that
// point's other FP32 blocks (on the 512-instance batch, orders <= 32 at 0.59
// of the FP64 time raised the re-factorisation pass from 4.6 to 8.0 ms and
// the evaluation from 21.2 to 22.7 ms; at 0.70 to 0.84 the re-factorised
// items rose from 121k to 677k; orders 33..96 at 0.28 to 0.42 gain).  Results
// do not depend on the choice beyond rounding; CGD_FLAG_NO_AUTOTUNE keeps the
// default shapes and the FP32 pass for every eligible class.
constexpr double kMixedFp32Gain = 0.5;
constexpr int64_t kTuneSample = 8192;
constexpr double kTuneTie = 0.02;

cgd_status autotune(cgd_ctx *c) {
    for (int k = 0; k < kRegClasses; ++k) c->reg_var[k] = 0;
    for (int k = 0; k < kMfmaClasses; ++k) c->mfma_var[k] = 0;
    c->tau_scale.assign(c->blocks.size(), 1.0);
    const std::string nlow = "\"lowrank_blocks\": " + std::to_string(c->lowrank_blocks) + ", ";
    if (c->flags & CGD_FLAG_NO_AUTOTUNE) {
        c->tune_json = "{\"autotune\": false, " + nlow + "\"classes\": []}";
        return make_lu_lists(c);
    }
    std::string rep = "{\"autotune\": true, " + nlow + "\"classes\": [";
    bool first = true;
    hipStream_t st = c->stream;
    const bool mixed = c->prec == CGD_PREC_MIXED;
    if (c->schur_nwg > 0)
        HIP_OK(launch_schur_build(c->d_schur, c->d_schur_prefix, (int)c->schur.size(), c->schur_nwg, c->schur_maxA,
                                  c->d_pool, c->d_eig, c->d_pool, c->d_pool32, st));
    int2 *d_items = nullptr;
    int *d_aux = nullptr;  // [0] list length, [1] status of the tuning launches
    HIP_OK(hipMalloc((void **)&d_items, sizeof(int2) * kTuneSample));
    HIP_OK(hipMalloc((void **)&d_aux, 2 * sizeof(int)));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    cgd_status result = CGD_OK;
    auto timed = [&](auto &&launch, double &ms) -> hipError_t {
        hipError_t e = launch();  // warm-up
        if (e != hipSuccess) return e;
        ms = 1e30;
        for (int rep_i = 0; rep_i < 3; ++rep_i) {
            if ((e = hipEventRecord(e0, st)) != hipSuccess) return e;
            if ((e = launch()) != hipSuccess) return e;
            if ((e = hipEventRecord(e1, st)) != hipSuccess) return e;
            if ((e = hipEventSynchronize(e1)) != hipSuccess) return e;
            float t = 0;
            if ((e = hipEventElapsedTime(&t, e0, e1)) != hipSuccess) return e;
            ms = std::min(ms, (double)t);
        }
        return hipSuccess;
    };
    for (int k = 0; k < kG64 && result == CGD_OK; ++k) {
        // this class's blocks; on the mixed path a class with FP32 blocks is
        // sampled over those only (the MFMA kernel takes orders up to its class limit)
        std::vector<int32_t> blk;
        int64_t total = 0;
        int maxn = 0;
        bool any32 = false;
        for (size_t b = 0; b < c->blocks.size(); ++b) {
            const BlockDev &d = c->blocks[b];
            if (!c->is_hess[b] && d.cls == k && mixed && d.fp32 && mfma_class_of(d.nb) == k) any32 = true;
        }
        for (size_t b = 0; b < c->blocks.size(); ++b) {
            const BlockDev &d = c->blocks[b];
            if (c->is_hess[b] || d.lowrank || d.cls != k) continue;
            if (any32 && !(d.fp32 && mfma_class_of(d.nb) == k)) continue;
            blk.push_back((int32_t)b);
            total += c->inst[d.inst].npts;
            maxn = std::max(maxn, d.nb);
        }
        if (total == 0) continue;
        // a class with density-mode blocks keeps to register-kernel shapes (they
        // write the trailing Schur complement the expansion reads)
        bool keeps = false;
        for (size_t b = 0; b < c->blocks.size(); ++b)
            if (!c->is_hess[b] && c->blocks[b].cls == k && c->blocks[b].nkeep) keeps = true;
        const int n64 = k < kRegClasses ? (keeps ? reg_kernel_variants(k) : reg_variants(k)) : 1;
        const int n32 = any32 ? mfma_variants(k) : 0;
        if (n64 < 2 && n32 == 0) continue;  // nothing to choose
        const int64_t S = std::min<int64_t>(total, kTuneSample);
        std::vector<int2> items(S);
        {
            size_t j = 0;
            int64_t base = 0;
            for (int64_t q = 0; q < S; ++q) {
                const int64_t t = q * total / S;
                while (base + c->inst[c->blocks[blk[j]].inst].npts <= t) base += c->inst[c->blocks[blk[j++]].inst].npts;
                items[q] = make_int2(blk[j], (int)(t - base));
            }
        }
        const int cnt[2] = {(int)S, 0};
        hipError_t e = hipMemcpy(d_items, items.data(), sizeof(int2) * S, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(d_aux, cnt, sizeof(cnt), hipMemcpyHostToDevice);
        LuLaunch a{nullptr, nullptr, 0, 0, d_items, d_aux, S, c->d_blocks, c->d_inst, c->d_pool, c->d_rb, c->d_eig,
                   c->d_contrib, d_aux + 1, c->d_tpool, c->d_tw};
        std::vector<double> t64(n64, -1.0), t32(n32, -1.0);
        for (int v = 0; v < n64 && e == hipSuccess; ++v)
            e = timed([&] { return k < kRegClasses ? launch_lu_reg(k, v, a, st)
                                                     : launch_lu_big(a, c->d_work, c->big_ldw, c->big_nwg, st); },
                      t64[v]);
        LuLaunch a32 = a;
        a32.pool = c->d_pool32;
        // the FP32 error model checked on the sample: each item's contribution
        // (the block's term of log G at the point) from the FP32 kernel against
        // the FP64 one, in units of the block's assumed relative error of G
        std::vector<double2> c64;
        if (n32 > 0 && e == hipSuccess) {
            c64.resize(c->ncontrib);
            e = hipMemcpy(c64.data(), c->d_contrib, sizeof(double2) * c->ncontrib, hipMemcpyDeviceToHost);
        }
        for (int v = 0; v < n32 && e == hipSuccess; ++v)
            e = timed([&] { return launch_lu_mfma(k, v, a32, st); }, t32[v]);
        double ratio32 = -1.0;
        if (n32 > 0 && e == hipSuccess) {
            std::vector<double2> c32(c->ncontrib);
            e = hipMemcpy(c32.data(), c->d_contrib, sizeof(double2) * c->ncontrib, hipMemcpyDeviceToHost);
            if (e == hipSuccess) {
                ratio32 = 0.0;
                for (const int2 &it : items) {
                    const BlockDev &d = c->blocks[it.x];
                    const InstDev &I = c->inst[d.inst];
                    const int64_t slot = I.c_off + (int64_t)it.y * I.nblocks + d.blk;
                    const double dx = c32[slot].x - c64[slot].x, dy = c32[slot].y - c64[slot].y;
                    const double tau_b = kTauScale * (d.nb + 1) * 5.9604644775390625e-08;
                    ratio32 = std::max(ratio32, std::sqrt(dx * dx + dy * dy) / tau_b);
                }
                // keep a margin of two over what the sample shows (the model's own
                // margin on the workloads that set it); the bound only ever grows
                const double scale = std::max(1.0, ratio32 / kTauMargin);
                for (int32_t b : blk) c->tau_scale[b] = scale;
            }
        }
        if (e != hipSuccess) {
            result = fail(CGD_ERR_DEVICE, std::string("autotune: ") + hipGetErrorString(e));
            break;
        }
        // the first variant within kTuneTie of the fastest: shapes that time alike
        // do not flip from one context (or run) to the next
        auto pick = [](const std::vector<double> &t) {
            const double best = *std::min_element(t.begin(), t.end());
            for (size_t v = 0; v < t.size(); ++v)
                if (t[v] <= best * (1.0 + kTuneTie)) return (int)v;
            return 0;
        };
        const int b64 = pick(t64);
        if (k < kRegClasses) c->reg_var[k] = b64;
        int b32 = -1;
        if (n32 > 0) {
            b32 = pick(t32);
            c->mfma_var[k] = b32;
        }
        const bool keep32 = n32 > 0 && t32[b32] < kMixedFp32Gain * t64[b64];
        if (n32 > 0 && !keep32)
            for (int32_t b : blk) c->blocks[b].fp32 = 0;
        std::string f64s, f32s;
        for (int v = 0; v < n64; ++v) {
            char buf[128];
            snprintf(buf, sizeof(buf), "%s\"%s\": %.4f", v ? ", " : "",
                     k < kRegClasses ? reg_variant_name(k, v) : "lu_big_f64", t64[v]);
            f64s += buf;
        }
        for (int v = 0; v < n32; ++v) {
            char buf[128];
            snprintf(buf, sizeof(buf), "%s\"%s\": %.4f", v ? ", " : "", mfma_variant_name(k, v), t32[v]);
            f32s += buf;
        }
        // no fixed-size buffer: the timing lists grow with the variants
        rep += std::string(first ? "" : ", ") + "{\"class\": " + std::to_string(k) +
               ", \"max_order\": " + std::to_string(maxn) + ", \"items\": " + std::to_string((long long)total) +
               ", \"sample\": " + std::to_string((long long)S) + ", \"fp64_ms\": {" + f64s + "}, \"fp32_ms\": {" +
               f32s + "}, " + (ratio32 >= 0.0 ? "\"fp32_err_ratio_max\": " + std::to_string(ratio32) + ", " : "") +
               "\"fp64_kernel\": \"" + (k < kRegClasses ? reg_variant_name(k, b64) : "lu_big_f64") +
               "\", \"fp32_kernel\": \"" + (keep32 ? mfma_variant_name(k, b32) : "") + "\", \"precision\": \"" +
               (keep32 ? "fp32+fp64" : "fp64") + "\"}";
        first = false;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(d_items);
    (void)hipFree(d_aux);
    if (result != CGD_OK) return result;
    c->tune_json = rep + "]}";
    // tau of each instance from the blocks left with an FP32 pass
    for (InstDev &I : c->inst) I.tau = 0.0;
    for (size_t b = 0; b < c->blocks.size(); ++b) {
        const BlockDev &d = c->blocks[b];
        if (d.fp32) c->inst[d.inst].tau += c->tau_scale[b] * kTauScale * (d.nb + 1) * 5.9604644775390625e-08;
    }
    HIP_OK(hipMemcpy(c->d_blocks, c->blocks.data(), sizeof(BlockDev) * c->blocks.size(), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(c->d_inst, c->inst.data(), sizeof(InstDev) * c->inst.size(), hipMemcpyHostToDevice));
    const cgd_status sl = make_lu_lists(c);
    if (sl != CGD_OK) return sl;
    lu_work(c);
    return CGD_OK;
}

cgd_status build(cgd_ctx *c, const cgd_instance *inst, int32_t n_inst) {
    std::vector<HostInst> hinst(n_inst);
    std::vector<HostBlock> hblocks;
    const bool dense = c->flags & CGD_FLAG_DENSE_INTERNAL;
    const bool use_schur = !(c->flags & CGD_FLAG_NO_SCHUR);
    const bool want_grad = c->flags & CGD_FLAG_GRAD;
    const bool lowrank_ok = !(c->flags & CGD_FLAG_NO_LOWRANK) && !want_grad;
    const bool moments = c->flags & (CGD_FLAG_MOMENTS | CGD_FLAG_CUMULANTS);
    if (moments && (want_grad || c->prec != CGD_PREC_FP64))
        return fail(CGD_ERR_ARG, "CGD_FLAG_MOMENTS / CGD_FLAG_CUMULANTS need CGD_PREC_FP64 and no CGD_FLAG_GRAD");
    if (dense)
        for (int i = 0; i < n_inst; ++i)
            if ((int64_t)inst[i].M * inst[i].K > 4096)
                return fail(CGD_ERR_ARG, "instance " + std::to_string(i) + ": M*K too large for CGD_FLAG_DENSE_INTERNAL");
    if (want_grad && dense)
        for (int i = 0; i < n_inst; ++i)
            if (inst[i].K > 1) return fail(CGD_ERR_ARG, "CGD_FLAG_GRAD works with internal-mode blocks (no CGD_FLAG_DENSE_INTERNAL)");
    // per instance (validation, assembly, auto grid, tail bound) on up to 16
    // host threads; results are merged in instance order
    struct InstOut {
        cgd_status st = CGD_OK;
        std::string err;
        std::vector<HostBlock> blocks;
        std::vector<GradHost> grads;
        HostInstCopy copy;
    };
    std::vector<InstOut> outs(n_inst);
    const double tol = c->tol;
    auto one = [&](int i) -> cgd_status {
        const cgd_instance &in = inst[i];
        InstOut &o = outs[i];
        cgd_status s = validate(in, i);
        if (s != CGD_OK) return s;
        if (in.distinguishable && want_grad)
            return fail(CGD_ERR_ARG, "instance " + std::to_string(i) + ": distinguishable inputs do not support CGD_FLAG_GRAD");
        HostInst &hi = hinst[i];
        hi.L = in.L;
        hi.nvar = 2 * (int)kept_fine_modes(in).size();
        hi.fock_n = hi.nvar ? in.fock_cutoff : 0;
        if (hi.nvar && (moments || want_grad || c->prec != CGD_PREC_FP64))
            return fail(CGD_ERR_ARG, "instance " + std::to_string(i) +
                                         ": kept modes need CGD_PREC_FP64 and no CGD_FLAG_GRAD / MOMENTS / CUMULANTS");
        for (int l = 0; l < in.L; ++l) {
            hi.N[l] = in.cutoff[l];
            hi.auto_grid[l] = in.grid && in.grid[l] == 0;
            hi.G[l] = hi.auto_grid[l] ? 0 : (in.grid ? in.grid[l] : in.cutoff[l] + 1);
            if (moments && (!in.grid || in.grid[l] == 0)) {
                // points on the circle in t: enough to keep the aliasing (rho / R)^G = 4^-G negligible
                hi.auto_grid[l] = false;
                hi.G[l] = std::max(kMomentPoints, 2 * (in.cutoff[l] + 1));
            }
        }
        // per internal mode squeezing: tanh^2 r_jk = (lambda_k / lambda_0) tanh^2 r_j;
        // fully distinguishable inputs (App. D): r_jk = r_j delta_jk
        std::vector<std::vector<double>> rk(in.M, std::vector<double>(in.K));
        for (int j = 0; j < in.M; ++j)
            for (int k = 0; k < in.K; ++k) {
                if (in.distinguishable) {
                    rk[j][k] = j == k ? in.r[j] : 0.0;
                    continue;
                }
                const double ratio = in.K == 1 ? 1.0 : in.schmidt[k] / in.schmidt[0];
                const double t = std::sqrt(ratio) * std::tanh(in.r[j]);
                if (!(t < 1.0)) return fail(CGD_ERR_NONPHYSICAL, "instance " + std::to_string(i) + ": Schmidt weights");
                rk[j][k] = std::atanh(t);
            }
        if (want_grad) {
            HostInstCopy &hc = o.copy;
            hc.M = in.M;
            hc.K = in.K;
            hc.T.resize((size_t)in.M * in.M);
            for (size_t e = 0; e < hc.T.size(); ++e) hc.T[e] = cx(in.T, e);
            hc.r.assign(in.r, in.r + in.M);
            if (in.schmidt) hc.schmidt.assign(in.schmidt, in.schmidt + in.K);
            if (in.alpha) {
                hc.alpha_v.resize(in.M);
                for (int j = 0; j < in.M; ++j) hc.alpha_v[j] = cx(in.alpha, j);
            }
            hc.rk = rk;
        }
        if (dense || in.K == 1) {
            std::vector<int> ks(in.K);
            for (int k = 0; k < in.K; ++k) ks[k] = k;
            s = assemble_block(in, i, ks, in.K > 1, use_schur, rk, hi, o.blocks, want_grad ? &o.grads : nullptr,
                               moments, lowrank_ok);
            if (s != CGD_OK) return s;
        } else {
            for (int k = 0; k < in.K; ++k) {
                s = assemble_block(in, i, {k}, false, use_schur, rk, hi, o.blocks, want_grad ? &o.grads : nullptr,
                                   moments, lowrank_ok);
                if (s != CGD_OK) return s;
            }
        }
        // grid entries 0: the smallest G_l >= N_l + 1 whose tail bound
        // Pr(b_l >= G_l) is at most tol / (10 L); then the wrap bound of the grid
        if (moments) {
            // circle radius in t a quarter of the distance to the nearest singularity,
            // |t| = log(1 / ||H||): there I - D(e^t) H stays accretive
            if (!(hi.hnorm < 1.0)) return fail(CGD_ERR_NONPHYSICAL, "instance " + std::to_string(i) + ": ||H|| >= 1");
            hi.rho = 0.25 * std::log(1.0 / std::max(hi.hnorm, 1e-300));
            hi.rho = std::min(hi.rho, 1.0);
            int gmin = 1 << 30;
            int64_t np2 = 1;
            for (int l = 0; l < in.L; ++l) {
                gmin = std::min(gmin, hi.G[l]);
                np2 *= hi.G[l];
                if (np2 > (int64_t)1 << 31) return fail(CGD_ERR_ARG, "instance " + std::to_string(i) + ": grid too large");
            }
            hi.wrap_bound = std::pow(0.25, gmin);  // relative aliasing scale of the Taylor coefficients
            for (int l = 0; l < in.L; ++l) std::vector<BinMarginal>().swap(hi.marg[l]);
            return CGD_OK;
        }
        bool any_auto = false;
        for (int l = 0; l < in.L; ++l) any_auto |= hi.auto_grid[l];
        if (any_auto && !(tol > 0.0 && std::isfinite(tol)))
            return fail(CGD_ERR_ARG, "instance " + std::to_string(i) + ": an automatic grid needs a finite tol > 0");
        const double target = std::log(tol / (10.0 * in.L));
        int64_t npts = 1;
        hi.wrap_bound = 0.0;
        for (int l = 0; l < in.L; ++l) {
            if (hi.auto_grid[l]) {
                int lo = hi.N[l] + 1, hi_g = lo;
                while (hi_g < 4096 && bin_log_tail(hi.marg[l], hi_g) > target) hi_g = std::min(4096, 2 * hi_g);
                if (bin_log_tail(hi.marg[l], hi_g) > target)
                    return fail(CGD_ERR_ARG, "instance " + std::to_string(i) + ": an automatic grid for bin " +
                                                 std::to_string(l) + " would exceed 4096 points");
                while (lo < hi_g) {  // smallest G in [lo, hi_g] meeting the target
                    const int mid = lo + (hi_g - lo) / 2;
                    if (bin_log_tail(hi.marg[l], mid) <= target) hi_g = mid; else lo = mid + 1;
                }
                hi.G[l] = hi_g;
            }
            hi.wrap_bound += std::exp(bin_log_tail(hi.marg[l], hi.G[l]));
            npts *= hi.G[l];
            if (npts > (int64_t)1 << 31) return fail(CGD_ERR_ARG, "instance " + std::to_string(i) + ": grid too large");
        }
        for (int l = 0; l < in.L; ++l) std::vector<BinMarginal>().swap(hi.marg[l]);
        return CGD_OK;
    };
    {
        std::atomic<int> next{0};
        auto work = [&]() {
            for (int i; (i = next.fetch_add(1)) < n_inst;) {
                const cgd_status st = one(i);
                if (st != CGD_OK) {
                    outs[i].st = st;
                    outs[i].err = g_err;
                }
            }
        };
        const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
        const int nthr = (int)std::min<int64_t>({(int64_t)16, (int64_t)hw, (int64_t)n_inst});
        std::vector<std::thread> pool;
        for (int t = 1; t < nthr; ++t) pool.emplace_back(work);
        work();
        for (auto &t : pool) t.join();
    }
    for (int i = 0; i < n_inst; ++i)
        if (outs[i].st != CGD_OK) {
            g_err = outs[i].err;
            return outs[i].st;
        }
    for (int i = 0; i < n_inst; ++i) {
        for (HostBlock &b : outs[i].blocks) hblocks.push_back(std::move(b));
        for (GradHost &g : outs[i].grads) c->grads.push_back(std::move(g));
        if (want_grad) {
            c->hinst_copy.push_back(std::move(outs[i].copy));
            HostInstCopy &hc = c->hinst_copy.back();
            hc.alpha = hc.alpha_v.empty() ? nullptr : hc.alpha_v.data();
        }
    }
    c->wrap_bound.resize(n_inst);
    c->grid_used.clear();
    for (int i = 0; i < n_inst; ++i) {
        c->wrap_bound[i] = hinst[i].wrap_bound;
        for (int l = 0; l < hinst[i].L; ++l) c->grid_used.push_back(hinst[i].G[l]);
    }

    // instances
    c->inst.resize(n_inst);
    c->prob_offsets.assign(n_inst + 1, 0);
    c->inst_pt_prefix.assign(n_inst, 0);
    int64_t pt = 0, co = 0, po = 0, ng = 0, tab = 0;
    c->dinst.clear();
    c->dprefix.clear();
    c->hprefix.clear();
    c->dnpts = c->htotal = c->nmat = 0;
    c->dens_lds = 0;
    for (int i = 0; i < n_inst; ++i) {
        InstDev &d = c->inst[i];
        std::memset(&d, 0, sizeof(d));
        const HostInst &h = hinst[i];
        d.L = h.L;
        d.nblocks = h.nblocks;
        int64_t np = 1, nprob = 1, ngi = 1;
        for (int l = 0; l < h.L; ++l) {
            d.G[l] = h.G[l];
            d.N[l] = h.N[l];
            nprob *= h.N[l] + 1;
            ngi *= h.G[l];
            if (l > 0) np *= h.G[l];
        }
        d.H1 = h.G[0] / 2 + 1;
        np *= d.H1;
        d.nvar = h.nvar;
        d.fock_n = h.fock_n;
        d.E = 1;
        for (int k = 0; k < h.nvar; ++k) d.E *= h.fock_n + 1;
        if (h.nvar) {
            if (np * d.E > ((int64_t)1 << 31))
                return fail(CGD_ERR_ARG, "instance " + std::to_string(i) + ": grid points times (fock_cutoff+1)^(2g) exceed 2^31");
            po += po & 1;  // complex output: even offset
            c->dinst.push_back(i);
            c->dprefix.push_back(c->dnpts);
            c->hprefix.push_back(c->nmat);
            c->dnpts += np;
            c->htotal += nprob * d.E;
            c->nmat += nprob;
            if (d.E <= kDensityLdsValues) c->dens_lds = std::max(c->dens_lds, d.E);
            nprob *= 2 * d.E;
        }
        d.gv_off = tab;
        // the region also holds the last DFT pass's complex output, prod (N_l + 1)
        // values per element, which can exceed the points (H1 < N_1 + 1)
        tab += (h.nvar ? std::max(np, nprob / (2 * d.E)) : np) * d.E;
        d.npts = np;
        d.pt_off = pt;
        d.c_off = co;
        d.prob_off = po;
        d.nprobs = nprob;
        d.logpr0_re = h.logpr0;
        d.logpr0_im = 0.0;
        d.rho = h.rho;
        d.dft_log = (c->flags & CGD_FLAG_CUMULANTS) ? 1 : 0;
        d.first_block = -1;
        d.tau = 0.0;
        c->inst_pt_prefix[i] = pt;
        c->prob_offsets[i] = po;
        pt += np;
        co += np * h.nblocks;
        po += nprob;
        ng += ngi;
    }
    c->prob_offsets[n_inst] = po;
    c->ntab = tab;
    c->npts = pt;
    c->ncontrib = co;
    c->nprobs = po;
    c->ngrid = ng;

    // pools and block descriptors
    std::vector<double2> pool;
    std::vector<int32_t> rbpool;
    std::vector<double> eigpool;
    auto push_mat = [&](const CMat &A) {
        const int64_t off = (int64_t)pool.size();
        for (const cplx &z : A.a) pool.push_back(make_double2(z.real(), z.imag()));
        return off;
    };
    c->blocks.resize(hblocks.size());
    c->is_hess.assign(hblocks.size(), 0);
    std::vector<int> hbins(hblocks.size(), -1), pbins(hblocks.size(), -1);
    const bool use_hess = choose_hessenberg(c, hblocks, hbins, pbins);
    std::vector<int32_t> permpool;
    for (size_t b = 0; b < hblocks.size(); ++b) {
        const HostBlock &h = hblocks[b];
        BlockDev &d = c->blocks[b];
        std::memset(&d, 0, sizeof(d));
        InstDev &I0 = c->inst[h.inst];
        if (I0.first_block < 0) I0.first_block = (int32_t)b;
        const int hbin = hbins[b];
        const bool hess = use_hess && hbin >= 0;
        c->is_hess[b] = hess;
        d.cls = kRegClasses;
        for (int k = 0; k < kRegClasses; ++k)
            if (h.nb <= reg_class_limit(k)) { d.cls = k; break; }
        // blocks of order 0 (one bin: eigenvalues only) have no factorisation to do in FP32
        d.fp32 = (!hess && c->prec == CGD_PREC_MIXED && h.nb > 0 && h.nb <= mfma_class_limit(kMfmaClasses - 1)) ? 1 : 0;
        if (d.fp32) {
            // relative error of an FP32 value of G: kTauScale (n + 1) 2^-24 per block, summed
            I0.tau += kTauScale * (h.nb + 1) * 5.9604644775390625e-08;
        }
        d.inst = h.inst;
        d.blk = h.blk;
        d.nb = h.nb;
        d.bordered = h.bordered;
        d.nkeep = h.nkeep;
        if (h.lowrank) {
            // no factorisation: its (L + 1) r x r matrices to the pool, its points to lowrank_points
            d.lowrank = h.lowrank;
            d.fp32 = 0;
            d.schur_axis = -1;
            d.lr_off = (int64_t)pool.size();
            for (const cplx &z : h.lr) pool.push_back(make_double2(z.real(), z.imag()));
            auto &lr = c->lowrank[h.lowrank - 1];
            if (lr.jobs.empty() || c->blocks[lr.blk[lr.jobs.back().x]].inst != h.inst)
                lr.jobs.push_back(make_int2((int)lr.blk.size(), 0));
            lr.blk.push_back((int32_t)b);
            lr.jobs.back().y++;
            c->lowrank_blocks++;
            continue;
        }
        if (h.nkeep) {
            if (d.cls >= kRegClasses)
                return fail(CGD_ERR_ARG, "instance " + std::to_string(h.inst) + ": a block with kept modes has order " +
                                             std::to_string(h.nb) + " > " + std::to_string(reg_class_limit(kRegClasses - 1)));
            const int nt = h.nkeep + h.bordered;
            d.t_off = c->ntpool;
            c->ntpool += I0.npts * nt * nt;
            d.kv_off = (int64_t)rbpool.size();
            rbpool.insert(rbpool.end(), h.kv.begin(), h.kv.end());
        }
        d.schur_axis = h.schur_axis;
        d.n_eig = (int32_t)h.eig.size();
        d.rb_off = (int64_t)rbpool.size();
        rbpool.insert(rbpool.end(), h.rowbin.begin(), h.rowbin.end());
        d.eig_off = (int64_t)eigpool.size();
        eigpool.insert(eigpool.end(), h.eig.begin(), h.eig.end());
        if (h.schur_axis >= 0) {
            SchurDev sj;
            std::memset(&sj, 0, sizeof(sj));
            const InstDev &I = c->inst[h.inst];
            sj.inst = h.inst;
            sj.axis = h.schur_axis;
            sj.nA = (int32_t)h.eig.size();
            sj.nB = h.nb;
            sj.nk = h.schur_axis == 0 ? I.H1 : I.G[h.schur_axis];
            sj.Gax = I.G[h.schur_axis];
            sj.p_off = push_mat(h.P);
            sj.q_off = push_mat(h.Q);
            sj.hbb_off = push_mat(h.H);
            sj.eig_off = d.eig_off;
            sj.rho = I.rho;
            const int64_t csize = (int64_t)sj.nk * h.nb * h.nb;
            sj.c_off = (int64_t)pool.size();
            pool.resize(pool.size() + csize, make_double2(0, 0));
            d.h_off = sj.c_off;
            d.hs_stride = (int64_t)h.nb * h.nb;
            if (h.nb > 0) {
                c->schur.push_back(sj);
                c->schur_maxA = std::max(c->schur_maxA, sj.nA);
            }
            if (hess) {
                HessDev hd;
                std::memset(&hd, 0, sizeof(hd));
                hd.inst = h.inst;
                hd.blk = h.blk;
                hd.n = h.nb;
                hd.axA = h.schur_axis;
                hd.axB = hbin;
                hd.axP = -1;
                hd.dP = 1;
                hd.dA = sj.nk;
                hd.dB = hbin == 0 ? I.H1 : I.G[hbin];
                hd.GA = I.G[h.schur_axis];
                hd.GB = I.G[hbin];
                hd.n_eig = d.n_eig;
                hd.c_off = sj.c_off;
                hd.eig_off = d.eig_off;
                hd.rho = I.rho;
                const int pbin = pbins[b];
                if (pbin >= 0) {
                    // pair route: rows of bin P first, S (rows of bin B) per pair after
                    // the uploaded pool (offsets relative to its end until it is known)
                    PairDev pd;
                    std::memset(&pd, 0, sizeof(pd));
                    pd.inst = h.inst;
                    pd.n = h.nb;
                    pd.perm_off = (int64_t)permpool.size();
                    for (int i = 0; i < h.nb; ++i)
                        if (h.rowbin[i] == pbin) permpool.push_back(i);
                    pd.nP = (int32_t)(permpool.size() - pd.perm_off);
                    for (int i = 0; i < h.nb; ++i)
                        if (h.rowbin[i] == hbin) permpool.push_back(i);
                    pd.axA = h.schur_axis;
                    pd.axP = pbin;
                    pd.dA = sj.nk;
                    pd.dP = pbin == 0 ? I.H1 : I.G[pbin];
                    pd.GA = I.G[h.schur_axis];
                    pd.GP = I.G[pbin];
                    pd.n_eig = d.n_eig;
                    pd.c_off = sj.c_off;
                    pd.hs_stride = (int64_t)h.nb * h.nb;
                    pd.eig_off = d.eig_off;
                    pd.rho = I.rho;
                    const int nH = h.nb - pd.nP;
                    pd.s_off = c->s_region;
                    c->s_region += (int64_t)pd.dA * pd.dP * nH * nH;
                    pd.ec_off = c->hess_nec;
                    c->pair_ldw = std::max(c->pair_ldw, h.nb);
                    c->pair_prefix.push_back(c->npairs);
                    c->npairs += (int64_t)pd.dA * pd.dP;
                    c->pairs.push_back(pd);
                    hd.n = nH;
                    hd.axP = pbin;
                    hd.dP = pd.dP;
                    hd.dA = pd.dA * pd.dP;
                    hd.n_eig = 0;
                    hd.c_off = pd.s_off;  // relative for now
                }
                hd.cls = 0;
                while (hd.n > hess_class_limit(hd.cls)) ++hd.cls;
                hd.t_off = c->hess_ntab;
                c->hess_ntab += (int64_t)hd.dA * hd.dB;
                hd.ec_off = c->hess_nec;
                c->hess_nec += hd.dA;
                c->hess_all.push_back(hd);
            }
        } else {
            d.h_off = push_mat(h.H);
            d.hs_stride = 0;
        }
    }
    // the S region of the pair route follows the uploaded pool
    c->pool_host = (int64_t)pool.size();
    for (PairDev &pd : c->pairs) pd.s_off += c->pool_host;
    for (HessDev &hd : c->hess_all)
        if (hd.axP >= 0) hd.c_off += c->pool_host;
    // schur work list: one workgroup per (job, k, row block)
    const int rows = schur_rows_per_wg();
    c->schur_prefix.clear();
    int64_t acc = 0;
    for (const SchurDev &s : c->schur) {
        c->schur_prefix.push_back(acc);
        acc += (int64_t)s.nk * ((s.nB + rows - 1) / rows);
    }
    c->schur_nwg = acc;
    if ((int64_t)c->schur_maxA * (1 + rows) * 16 > 150 * 1024)
        return fail(CGD_ERR_ARG, "eliminated bin too large for the Schur build");

    // LU work lists: FP64 groups (everything on the FP64 path; on the mixed path
    // the blocks without an FP32 pass), FP32 MFMA groups (mixed first pass),
    // and the capacity of the mixed second-pass lists per FP64 group
    for (int k = 0; k < kG64; ++k) c->g64[k].cls = k;
    for (int k = 0; k < kMfmaClasses; ++k) c->g32[k].cls = k;
    for (const HessDev &hd : c->hess_all) {
        HessClass &hc = c->hcls[hd.cls];
        hc.rprefix.push_back(hc.rnwg);
        hc.dprefix.push_back(hc.dnwg);
        hc.jobs.push_back(hd);
        hc.rnwg += hd.dA;
        hc.dnwg += (int64_t)hd.dA * ((hd.dB + 15) / 16);
        c->hess_sprefix.push_back(c->hess_spts);
        c->hess_spts += c->inst[hd.inst].npts;
    }
    {
        const cgd_status sl = make_lu_lists(c);
        if (sl != CGD_OK) return sl;
    }

    // DFT stages; twiddles exp(-2 pi i m / G) for every grid extent in use
    int Lmax = 0;
    for (auto &d : c->inst) Lmax = std::max(Lmax, d.L);
    {
        std::vector<double2> tw;
        for (InstDev &I : c->inst)
            for (int l = 0; l < I.L; ++l) {
                const int G = I.G[l];
                if (!c->tw_of.count(G)) {
                    c->tw_of[G] = (int64_t)tw.size();
                    for (int m = 0; m < G; ++m) {
                        const double a = -2.0 * M_PI * (double)m / (double)G;
                        tw.push_back(make_double2(std::cos(a), std::sin(a)));
                    }
                }
                I.tw_off[l] = (int32_t)c->tw_of[G];  // the LU kernels read their roots of unity here
            }
        cgd_status s;
        if ((s = upload(&c->d_tw, tw)) != CGD_OK) return s;
    }
    c->stages.resize(Lmax);
    for (int s = 0; s < Lmax; ++s) {
        DftStage &st = c->stages[s];
        for (int i = 0; i < n_inst; ++i) {
            const InstDev &I = c->inst[i];
            if (I.L <= s) continue;
            const int a = I.L - 1 - s;
            int64_t dims[kMaxBins];
            for (int l = 0; l < I.L; ++l) dims[l] = l <= a ? (l == 0 ? I.H1 : I.G[l]) : (I.N[l] + 1);
            DftStageDev d;
            std::memset(&d, 0, sizeof(d));
            d.inst = i;
            d.K = (int32_t)dims[a];
            d.Bout = I.N[a] + 1;
            d.G = I.G[a];
            d.tw_off = c->tw_of.at(d.G);
            d.final_stage = a == 0;
            d.outer = 1;
            for (int l = 0; l < a; ++l) d.outer *= dims[l];
            d.inner = I.E;  // density mode: every matrix element is a DFT of its own
            for (int l = a + 1; l < I.L; ++l) d.inner *= dims[l];
            d.in_off = I.gv_off;
            d.out_off = (a == 0 && !I.nvar) ? I.prob_off : I.gv_off;
            d.density = I.nvar ? 1 : 0;
            double gprod = 1;
            for (int l = 0; l < I.L; ++l) gprod *= I.G[l];
            d.scale = 1.0 / gprod;
            d.moments = I.rho > 0.0 ? 1 : 0;
            d.rho = I.rho;
            if (d.K <= kDftColsK) {
                st.cprefix.push_back(st.ctotal);
                st.ctotal += d.outer * d.inner;
                st.cdesc.push_back(d);
            } else {
                st.prefix.push_back(st.total);
                st.total += d.outer * d.Bout * d.inner;
                st.desc.push_back(d);
            }
        }
    }

    // algorithmic work per evaluation
    lu_work(c);
    for (const SchurDev &sj : c->schur) c->work_flops[CGD_STAGE_SCHUR] += 8.0 * sj.nA * (double)sj.nB * sj.nB * sj.nk;
    for (const HessDev &hd : c->hess_all) {
        // reduction: column k with m = n - k - 1 rows below the diagonal costs
        // 2 m (m + 1) complex multiply-adds for w and the left update and 2 n m for y
        // and the right update; factorisation: 2 (n - k - 1) per step
        double red = 0, fac = 0;
        for (int k = 0; k + 2 < hd.n; ++k) {
            const double m = hd.n - k - 1;
            red += 2.0 * m * (m + 1) + 2.0 * hd.n * m;
        }
        for (int k = 0; k + 1 < hd.n; ++k) fac += 2.0 * (hd.n - k - 1);
        c->work_flops[CGD_STAGE_HESS] += 8.0 * red * hd.dA;
        c->work_flops[CGD_STAGE_HESS_DET] += 8.0 * fac * (double)hd.dA * hd.dB;
    }
    for (const PairDev &pd : c->pairs) {
        double f = 0;  // the nP pivots of a partial LU of order n
        for (int k = 0; k < pd.nP; ++k) {
            const double m = pd.n - k - 1;
            f += 8.0 * m * m + 6.0 * m;
        }
        c->work_flops[CGD_STAGE_PAIR] += f * pd.dA * pd.dP;
    }
    for (const DftStage &st : c->stages) {
        for (const DftStageDev &d : st.desc) c->work_flops[CGD_STAGE_DFT] += 8.0 * d.outer * d.Bout * d.inner * d.K;
        for (const DftStageDev &d : st.cdesc) c->work_flops[CGD_STAGE_DFT] += 8.0 * d.outer * d.Bout * d.inner * d.K;
    }
    c->work_bytes[CGD_STAGE_DFT] = 16.0 * c->ntab + 8.0 * c->nprobs;
    for (int j : c->dinst) {
        // per value: one complex multiply for l, one per later position, of the
        // recurrence (about 1 + nvar / 2 on average); rho = R + R^H: one add
        const InstDev &I = c->inst[j];
        c->work_flops[CGD_STAGE_DENSITY] += 8.0 * (1.0 + 0.5 * I.nvar) * (double)I.npts * (double)I.E;
        c->work_bytes[CGD_STAGE_DENSITY] += 16.0 * (double)I.npts * (double)I.E;
    }
    c->work_flops[CGD_STAGE_DENSITY] += 2.0 * (double)c->htotal;
    c->work_bytes[CGD_STAGE_DENSITY] += 48.0 * (double)c->htotal;
    c->work_bytes[CGD_STAGE_COMBINE] = 16.0 * (c->ncontrib + 2 * c->npts);

    // uploads
    cgd_status s;
    if ((s = upload(&c->d_inst, c->inst)) != CGD_OK) return s;
    if ((s = upload(&c->d_blocks, c->blocks)) != CGD_OK) return s;
    if ((s = upload(&c->d_schur, c->schur)) != CGD_OK) return s;
    if ((s = upload(&c->d_schur_prefix, c->schur_prefix)) != CGD_OK) return s;
    if ((s = upload(&c->d_inst_pt_prefix, c->inst_pt_prefix)) != CGD_OK) return s;
    HIP_OK(hipMalloc((void **)&c->d_pool, sizeof(double2) * std::max<int64_t>(1, c->pool_host + c->s_region)));
    if (!pool.empty())
        HIP_OK(hipMemcpy(c->d_pool, pool.data(), sizeof(double2) * pool.size(), hipMemcpyHostToDevice));
    if (c->npairs > 0) {
        if ((s = upload(&c->d_pairs, c->pairs)) != CGD_OK) return s;
        if ((s = upload(&c->d_pair_prefix, c->pair_prefix)) != CGD_OK) return s;
        if ((s = upload(&c->d_perm, permpool)) != CGD_OK) return s;
        int ncu = 0, dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0)
            ncu = 256;
        c->pair_nwg = (int)std::min<int64_t>(c->npairs, 2 * (int64_t)ncu);
        HIP_OK(hipMalloc((void **)&c->d_pair_work,
                         sizeof(double2) * (size_t)c->pair_nwg * c->pair_ldw * c->pair_ldw));
    }
    if ((s = upload(&c->d_rb, rbpool)) != CGD_OK) return s;
    if ((s = upload(&c->d_eig, eigpool)) != CGD_OK) return s;
    for (int r = 1; r <= kLowRankMax; ++r) {
        auto &lr = c->lowrank[r - 1];
        for (const int2 &j : lr.jobs) {  // tiles of 16 blocks x a run of points
            lr.prefix.push_back(lr.ntiles);
            const InstDev &I = c->inst[c->blocks[lr.blk[j.x]].inst];
            const int64_t run = lowrank_points_per_tile();
            lr.ntiles += ((I.npts + run - 1) / run) * ((j.y + 15) / 16);
            lr.wstride = std::max(lr.wstride, I.L);
            lr.gstride = std::max(lr.gstride, (I.L + 1) * r * r);
        }
        if ((s = upload(&lr.d_blk, lr.blk)) != CGD_OK) return s;
        if ((s = upload(&lr.d_jobs, lr.jobs)) != CGD_OK) return s;
        if ((s = upload(&lr.d_prefix, lr.prefix)) != CGD_OK) return s;
    }
    for (auto &st : c->stages) {
        if ((s = upload(&st.d_desc, st.desc)) != CGD_OK) return s;
        if ((s = upload(&st.d_prefix, st.prefix)) != CGD_OK) return s;
        if ((s = upload(&st.d_cdesc, st.cdesc)) != CGD_OK) return s;
        if ((s = upload(&st.d_cprefix, st.cprefix)) != CGD_OK) return s;
    }
    if (!c->hess_all.empty()) {
        for (auto &hc : c->hcls) {
            if ((s = upload(&hc.d_jobs, hc.jobs)) != CGD_OK) return s;
            if ((s = upload(&hc.d_rprefix, hc.rprefix)) != CGD_OK) return s;
            if ((s = upload(&hc.d_dprefix, hc.dprefix)) != CGD_OK) return s;
        }
        if ((s = upload(&c->d_hess_all, c->hess_all)) != CGD_OK) return s;
        if ((s = upload(&c->d_hess_sprefix, c->hess_sprefix)) != CGD_OK) return s;
        HIP_OK(hipMalloc((void **)&c->d_eigc, sizeof(double2) * c->hess_nec));
        HIP_OK(hipMalloc((void **)&c->d_htable, sizeof(double2) * c->hess_ntab));
    }
    const int64_t nc = std::max<int64_t>(c->ncontrib, 1), np = std::max<int64_t>(c->npts, 1);
    const int64_t ntab = std::max<int64_t>(c->ntab, 1);
    HIP_OK(hipMalloc((void **)&c->d_contrib, sizeof(double2) * nc));
    HIP_OK(hipMalloc((void **)&c->d_logg, sizeof(double2) * np));
    HIP_OK(hipMalloc((void **)&c->d_gA, sizeof(double2) * ntab));
    HIP_OK(hipMalloc((void **)&c->d_gB, sizeof(double2) * ntab));
    HIP_OK(hipMalloc((void **)&c->d_tpool, sizeof(double2) * std::max<int64_t>(c->ntpool, 1)));
    if (!c->dinst.empty()) {
        if ((s = upload(&c->d_dinst, c->dinst)) != CGD_OK) return s;
        if ((s = upload(&c->d_dprefix, c->dprefix)) != CGD_OK) return s;
        if ((s = upload(&c->d_hprefix, c->hprefix)) != CGD_OK) return s;
    }
    HIP_OK(hipMalloc((void **)&c->d_status, sizeof(int)));
    HIP_OK(hipMemset(c->d_status, 0, sizeof(int)));
    HIP_OK(hipHostMalloc((void **)&c->h_status, sizeof(int), hipHostMallocDefault));
    *c->h_status = 0;
    HIP_OK(hipEventCreateWithFlags(&c->ev_status, hipEventDisableTiming));
    if (c->big_nwg > 0) {
        HIP_OK(hipMalloc((void **)&c->d_work, sizeof(double2) * (size_t)c->big_nwg * c->big_ldw * c->big_ldw));
    }
    if (c->prec == CGD_PREC_MIXED) {
        std::vector<float2> p32(pool.size());
        for (size_t i = 0; i < pool.size(); ++i) {
            p32[i].x = (float)pool[i].x;
            p32[i].y = (float)pool[i].y;
        }
        if ((s = upload(&c->d_pool32, p32)) != CGD_OK) return s;
        HIP_OK(hipMalloc((void **)&c->d_logg32, sizeof(double2) * np));
        HIP_OK(hipMalloc((void **)&c->d_counts, sizeof(int) * kG64));
        HIP_OK(hipMalloc((void **)&c->d_hist, sizeof(unsigned long long) * (size_t)n_inst * kMixedBuckets));
        HIP_OK(hipMalloc((void **)&c->d_cut, sizeof(int) * n_inst));
    }
    HIP_OK(prepare_kernels(c->big_nwg > 0 ? c->big_ldw : 0, c->schur_maxA, c->npairs > 0 ? c->pair_ldw : 0));
    // kernel variant (and, on the mixed path, precision) per size class, from
    // timings on this context's own work; then the work lists
    if ((s = autotune(c)) != CGD_OK) return s;
    if ((s = upload_lu_lists(c)) != CGD_OK) return s;
    if (want_grad) {
        cgd_status sg = build_grad(c, n_inst);
        if (sg != CGD_OK) return sg;
    }
    HIP_OK(hipDeviceSynchronize());
    return CGD_OK;
}

}  // namespace

extern "C" {

cgd_status cgd_create(cgd_ctx **out, const cgd_instance *inst, int32_t n_inst, cgd_precision prec, double tol,
                      uint32_t flags, void *hip_stream) {
    if (!out) return fail(CGD_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!inst || n_inst <= 0) return fail(CGD_ERR_ARG, "need at least one instance");
    if (prec != CGD_PREC_FP64 && prec != CGD_PREC_MIXED) return fail(CGD_ERR_ARG, "unknown precision");
    if (prec == CGD_PREC_MIXED && !(tol > 0)) return fail(CGD_ERR_ARG, "mixed precision needs tol > 0");
    if (flags & ~(CGD_FLAG_DENSE_INTERNAL | CGD_FLAG_NO_SCHUR | CGD_FLAG_GRAD | CGD_FLAG_HESSENBERG |
                  CGD_FLAG_NO_HESSENBERG | CGD_FLAG_NO_AUTOTUNE | CGD_FLAG_MOMENTS | CGD_FLAG_CUMULANTS |
                  CGD_FLAG_NO_LOWRANK))
        return fail(CGD_ERR_ARG, "unknown flags");
    if ((flags & CGD_FLAG_MOMENTS) && (flags & CGD_FLAG_CUMULANTS))
        return fail(CGD_ERR_ARG, "CGD_FLAG_MOMENTS and CGD_FLAG_CUMULANTS together");
    if ((flags & CGD_FLAG_HESSENBERG) && (flags & CGD_FLAG_NO_HESSENBERG))
        return fail(CGD_ERR_ARG, "CGD_FLAG_HESSENBERG and CGD_FLAG_NO_HESSENBERG together");
    cgd_ctx *c = new (std::nothrow) cgd_ctx();
    if (!c) return fail(CGD_ERR_NOMEM, "host allocation");
    c->n_inst = n_inst;
    c->prec = prec;
    c->tol = tol;
    c->flags = flags;
    c->stream = (hipStream_t)hip_stream;
    // validation errors come back from build before any device call
    cgd_status s = build(c, inst, n_inst);
    if (s == CGD_OK && hipGetDevice(&c->device) != hipSuccess) s = fail(CGD_ERR_DEVICE, "hipGetDevice failed");
    if (s == CGD_OK) {
        // the device address of cgd_eval_static's scratch array, once per device
        const hipError_t e = static_scratch_setup(c->device);
        if (e != hipSuccess) s = fail(CGD_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    if (s != CGD_OK) {
        free_ctx(c);
        return s;
    }
    *out = c;
    return CGD_OK;
}

cgd_status cgd_layout(const cgd_ctx *ctx, int64_t *n_probs_total, int64_t *prob_offsets, int64_t *n_grid_total) {
    if (!ctx) return fail(CGD_ERR_ARG, "ctx is NULL");
    if (n_probs_total) *n_probs_total = ctx->nprobs;
    if (prob_offsets)
        for (int i = 0; i <= ctx->n_inst; ++i) prob_offsets[i] = ctx->prob_offsets[i];
    if (n_grid_total) *n_grid_total = ctx->ngrid;
    return CGD_OK;
}

int64_t cgd_points(const cgd_ctx *ctx) { return ctx ? ctx->npts : 0; }

namespace {
// Device buffers one evaluation writes and reads back (all of them rewritten by
// every evaluation before they are read): the context's own (cgd_eval) or
// slices of the static per-device scratch (cgd_eval_static).
struct EvalBufs {
    double2 *contrib, *logg, *gA, *gB, *logg32, *eigc, *htable;
    int *counts, *cut;
    unsigned long long *hist;
    int2 *list;
    double2 *tpool;
};

EvalBufs ctx_bufs(const cgd_ctx *c) {
    return EvalBufs{c->d_contrib, c->d_logg, c->d_gA, c->d_gB, c->d_logg32, c->d_eigc, c->d_htable,
                    c->d_counts, c->d_cut, c->d_hist, c->d_list, c->d_tpool};
}

// Byte sizes of the EvalBufs fields in field order (0: not used by this context).
constexpr int kEvalBufs = 12;
void eval_buf_sizes(const cgd_ctx *c, size_t (&sz)[kEvalBufs]) {
    const bool mixed = c->prec == CGD_PREC_MIXED;
    const bool hess = !c->hess_all.empty();
    const size_t cz = sizeof(double2);
    const size_t v[kEvalBufs] = {cz * (size_t)c->ncontrib, cz * (size_t)c->npts, cz * (size_t)c->ntab,
                                 cz * (size_t)c->ntab, mixed ? cz * (size_t)c->npts : 0,
                                 hess ? cz * (size_t)c->hess_nec : 0, hess ? cz * (size_t)c->hess_ntab : 0,
                                 mixed ? sizeof(int) * kG64 : 0, mixed ? sizeof(int) * (size_t)c->n_inst : 0,
                                 mixed ? sizeof(unsigned long long) * (size_t)c->n_inst * kMixedBuckets : 0,
                                 mixed ? sizeof(int2) * (size_t)c->list_total : 0, cz * (size_t)c->ntpool};
    for (int i = 0; i < kEvalBufs; ++i) sz[i] = v[i];
}

// Enqueue every launch of one evaluation on stream st.
cgd_status enqueue_eval(cgd_ctx *c, hipStream_t st, double *d_probs, double *d_err_bound, const EvalBufs &b) {
    // mark(stage, 0) opens a timed span, mark(stage, 1) closes it
    auto mark = [&](int stage, int which) -> hipError_t {
        if (!c->timing) return hipSuccess;
        c->stage_ran[stage] = true;
        if (which == 0) {
            const size_t k = c->tev_stage.size();
            while (c->tev.size() < 2 * (k + 1)) {
                hipEvent_t e;
                const hipError_t err = hipEventCreate(&e);
                if (err != hipSuccess) return err;
                c->tev.push_back(e);
            }
            c->tev_stage.push_back(stage);
            c->tev_open = k;
            return hipEventRecord(c->tev[2 * k], st);
        }
        return hipEventRecord(c->tev[2 * c->tev_open + 1], st);
    };
    for (int i = 0; i < CGD_NSTAGES; ++i) c->stage_ran[i] = false;
    c->tev_stage.clear();
    if (c->schur_nwg > 0) {
        HIP_OK(mark(CGD_STAGE_SCHUR, 0));
        HIP_OK(launch_schur_build(c->d_schur, c->d_schur_prefix, (int)c->schur.size(), c->schur_nwg,
                                  c->schur_maxA, c->d_pool, c->d_eig, c->d_pool, c->d_pool32, st));
        HIP_OK(mark(CGD_STAGE_SCHUR, 1));
    }
    if (c->npairs > 0) {
        HIP_OK(mark(CGD_STAGE_PAIR, 0));
        HIP_OK(launch_pair_schur(c->d_pairs, c->d_pair_prefix, (int)c->pairs.size(), c->npairs, c->pair_nwg,
                                 c->d_pool, c->d_perm, c->d_eig, c->d_pair_work, c->pair_ldw, b.eigc,
                                 c->d_status, st));
        HIP_OK(mark(CGD_STAGE_PAIR, 1));
    }
    if (!c->hess_all.empty()) {
        HIP_OK(mark(CGD_STAGE_HESS, 0));
        for (auto &hc : c->hcls)
            HIP_OK(launch_hess_reduce((int)(&hc - c->hcls), hc.d_jobs, hc.d_rprefix, (int)hc.jobs.size(), hc.rnwg,
                                      c->d_pool, c->d_eig, b.eigc, st));
        HIP_OK(mark(CGD_STAGE_HESS, 1));
        HIP_OK(mark(CGD_STAGE_HESS_DET, 0));
        for (auto &hc : c->hcls)
            HIP_OK(launch_hess_det((int)(&hc - c->hcls), hc.d_jobs, hc.d_dprefix, (int)hc.jobs.size(), hc.dnwg,
                                   c->d_pool, b.eigc, b.htable, c->d_status, st));
        HIP_OK(launch_hess_scatter(c->d_hess_all, c->d_hess_sprefix, (int)c->hess_all.size(), c->hess_spts,
                                   c->d_inst, b.htable, b.contrib, st));
        HIP_OK(mark(CGD_STAGE_HESS_DET, 1));
    }
    const bool mixed = c->prec == CGD_PREC_MIXED;
    // timing: a slot spans from its first launch to its last one in this evaluation
    auto mark_begin = [&](int stage) -> hipError_t { return mark(stage, 0); };
    auto launch64 = [&](int k, const int2 *list, const int *count, int64_t cap) -> hipError_t {
        const LuClass &g = c->g64[k];
        LuLaunch a{g.d_jobs, g.d_prefix, (int)g.jobs.size(), g.nitems, list, count, cap, c->d_blocks,
                   c->d_inst, c->d_pool, c->d_rb, c->d_eig, b.contrib, c->d_status, b.tpool, c->d_tw,
                   list ? nullptr : g.d_hint};
        return k < kRegClasses ? launch_lu_reg(k, c->reg_var[k], a, st)
                               : launch_lu_big(a, c->d_work, c->big_ldw, c->big_nwg, st);
    };
    if (c->lowrank_blocks > 0) {
        // low-rank blocks: FP64 in both paths, no second pass
        HIP_OK(mark_begin(lu_stage(0)));
        for (int r = 1; r <= kLowRankMax; ++r) {
            const auto &lr = c->lowrank[r - 1];
            if (lr.ntiles == 0) continue;
            HIP_OK(launch_lowrank_points(r, lr.d_jobs, lr.d_prefix, (int)lr.jobs.size(), lr.ntiles, lr.d_blk,
                                         c->d_blocks, c->d_inst, c->d_pool, c->d_tw, b.contrib, c->d_status,
                                         lr.gstride, lr.wstride, st));
        }
        HIP_OK(mark(lu_stage(0), 1));
    }
    if (mixed)
        for (auto &g : c->g32) {
            if (g.nitems == 0) continue;
            LuLaunch a{g.d_jobs, g.d_prefix, (int)g.jobs.size(), g.nitems, nullptr, nullptr, 0, c->d_blocks,
                       c->d_inst, c->d_pool32, c->d_rb, c->d_eig, b.contrib, c->d_status, b.tpool, c->d_tw,
                       g.d_hint};
            HIP_OK(mark_begin(lu_stage(g.cls)));
            HIP_OK(launch_lu_mfma(g.cls, c->mfma_var[g.cls], a, st));
            HIP_OK(mark(lu_stage(g.cls), 1));
        }
    for (int k = 0; k < kG64; ++k) {
        const bool one = k == 0 && c->g64one.nitems > 0;
        if (c->g64[k].nitems == 0 && !one) continue;
        HIP_OK(mark_begin(lu_stage(k)));
        if (c->g64[k].nitems > 0) HIP_OK(launch64(k, nullptr, nullptr, 0));
        if (one) {
            const LuClass &g = c->g64one;
            LuLaunch a{g.d_jobs, g.d_prefix, (int)g.jobs.size(), g.nitems, nullptr, nullptr, 0, c->d_blocks,
                       c->d_inst, c->d_pool, c->d_rb, c->d_eig, b.contrib, c->d_status, b.tpool, c->d_tw, g.d_hint};
            HIP_OK(launch_lu_one_tile(a, st));
        }
        HIP_OK(mark(lu_stage(k), 1));
    }
    HIP_OK(mark(CGD_STAGE_COMBINE, 0));
    if (mixed) {
        // FP32 values -> select the points that matter -> FP64 re-factorisation of those
        HIP_OK(launch_combine(c->d_inst, c->d_inst_pt_prefix, c->n_inst, c->npts, b.contrib, b.logg32,
                              b.gA, st));
        HIP_OK(mark(CGD_STAGE_COMBINE, 1));
        HIP_OK(mark(CGD_STAGE_FIX, 0));
        HIP_OK(launch_zero_ints(b.counts, kG64, st));
        HIP_OK(launch_mixed_cut(c->d_inst, c->d_inst_pt_prefix, c->n_inst, c->npts, b.logg32, c->tol, b.hist,
                                b.cut, st));
        HIP_OK(launch_select_points(c->d_inst, c->d_inst_pt_prefix, c->n_inst, c->npts, c->d_blocks, b.logg32,
                                    b.cut, b.list, c->d_list_off, b.counts, kG64, st));
        for (int k = 0; k < kG64; ++k) {
            if (c->list_cap[k] == 0) continue;
            HIP_OK(launch64(k, b.list + c->list_off[k], b.counts + k, c->list_cap[k]));
        }
        HIP_OK(launch_combine(c->d_inst, c->d_inst_pt_prefix, c->n_inst, c->npts, b.contrib, b.logg, b.gA,
                              st));
        HIP_OK(mark(CGD_STAGE_FIX, 1));
    } else {
        HIP_OK(launch_combine(c->d_inst, c->d_inst_pt_prefix, c->n_inst, c->npts, b.contrib, b.logg, b.gA,
                              st));
        HIP_OK(mark(CGD_STAGE_COMBINE, 1));
    }
    if (c->dnpts > 0) {
        HIP_OK(mark(CGD_STAGE_DENSITY, 0));
        HIP_OK(launch_density_expand(c->d_inst, c->d_dinst, c->d_dprefix, (int)c->dinst.size(), c->dnpts,
                                     c->dens_lds, c->d_blocks, c->d_rb, b.contrib, b.tpool, b.logg, b.gA, st));
        HIP_OK(mark(CGD_STAGE_DENSITY, 1));
    }
    HIP_OK(mark(CGD_STAGE_DFT, 0));
    for (size_t si = 0; si < c->stages.size(); ++si) {
        DftStage &S = c->stages[si];
        const double2 *in = (si % 2 == 0) ? b.gA : b.gB;
        double2 *out = (si % 2 == 0) ? b.gB : b.gA;
        HIP_OK(launch_dft_cols(S.d_cdesc, S.d_cprefix, (int)S.cdesc.size(), S.ctotal, c->d_tw, in, out, d_probs,
                               mixed ? nullptr : d_err_bound, c->d_status, st));
        HIP_OK(launch_dft_stage(S.d_desc, S.d_prefix, (int)S.desc.size(), S.total, c->d_tw, in, out, d_probs,
                                mixed ? nullptr : d_err_bound, c->d_status, st));
    }
    HIP_OK(mark(CGD_STAGE_DFT, 1));
    if (c->htotal > 0) {
        HIP_OK(mark(CGD_STAGE_DENSITY, 0));
        HIP_OK(launch_density_hermitize(c->d_inst, c->d_dinst, c->d_hprefix, (int)c->dinst.size(), c->nmat,
                                        c->dens_lds, b.gA, b.gB, d_probs, st));
        HIP_OK(mark(CGD_STAGE_DENSITY, 1));
    }
    if (mixed) HIP_OK(launch_mixed_err(c->d_inst, c->n_inst, b.logg32, b.cut, d_err_bound, c->d_status, st));
    return CGD_OK;
}
}  // namespace

cgd_status cgd_eval(cgd_ctx *c, double *d_probs, double *d_err_bound) {
    if (!c) return fail(CGD_ERR_ARG, "ctx is NULL");
    if (!d_probs) return fail(CGD_ERR_ARG, "d_probs is NULL");
    cgd_status s = check_status(c);
    if (s != CGD_OK) return s;
    if (c->timing) {
        // per-stage events need the launches on the caller's stream, one by one
        s = enqueue_eval(c, c->stream, d_probs, d_err_bound, ctx_bufs(c));
        if (s != CGD_OK) return s;
    } else {
        // the launch sequence is captured once on a private stream into a HIP
        // graph and replayed on the caller's stream; captured again when the
        // output pointers change
        if (!c->gexec || c->g_probs != d_probs || c->g_err != d_err_bound) {
            if (c->gexec) { (void)hipGraphExecDestroy(c->gexec); c->gexec = nullptr; }
            if (!c->cap_stream) HIP_OK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
            HIP_OK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
            s = enqueue_eval(c, c->cap_stream, d_probs, d_err_bound, ctx_bufs(c));
            hipGraph_t graph = nullptr;
            const hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
            if (s != CGD_OK) { if (graph) (void)hipGraphDestroy(graph); return s; }
            if (e != hipSuccess) return fail(CGD_ERR_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
            const hipError_t e2 = hipGraphInstantiate(&c->gexec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e2 != hipSuccess) return fail(CGD_ERR_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e2));
            c->g_probs = d_probs;
            c->g_err = d_err_bound;
        }
        HIP_OK(hipGraphLaunch(c->gexec, c->stream));
    }
    HIP_OK(hipMemcpyAsync(c->h_status, c->d_status, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipEventRecord(c->ev_status, c->stream));
    c->status_pending = true;
    c->evaluated = true;
    c->last_static = false;
    return CGD_OK;
}

cgd_status cgd_eval_static(cgd_ctx *c, double *d_probs, double *d_err_bound) {
    if (!c) return fail(CGD_ERR_ARG, "ctx is NULL");
    if (!d_probs) return fail(CGD_ERR_ARG, "d_probs is NULL");
    cgd_status s = check_status(c);
    if (s != CGD_OK) return s;
    int dev = -1;
    HIP_OK(hipGetDevice(&dev));
    if (dev != c->device) return fail(CGD_ERR_ARG, "cgd_eval_static: the context's device is not the current device");
    unsigned char *base = (unsigned char *)static_scratch(dev);
    if (!base) return fail(CGD_ERR_STATE, "cgd_eval_static: no static scratch on this device");
    // slices of the static scratch, 256-byte aligned, in EvalBufs field order
    size_t sz[kEvalBufs];
    eval_buf_sizes(c, sz);
    void *ptr[kEvalBufs] = {};
    size_t off = 0;
    for (int i = 0; i < kEvalBufs; ++i) {
        if (sz[i] == 0) continue;
        ptr[i] = base + off;
        off += (sz[i] + 255) & ~(size_t)255;
    }
    if (off > kStaticScratchBytes)
        return fail(CGD_ERR_ARG, "cgd_eval_static: this context needs " + std::to_string(off) +
                                     " bytes of scratch, more than the " + std::to_string(kStaticScratchBytes) +
                                     " bytes of the static array");
    const EvalBufs b{(double2 *)ptr[0], (double2 *)ptr[1], (double2 *)ptr[2], (double2 *)ptr[3], (double2 *)ptr[4],
                     (double2 *)ptr[5], (double2 *)ptr[6], (int *)ptr[7], (int *)ptr[8],
                     (unsigned long long *)ptr[9], (int2 *)ptr[10], (double2 *)ptr[11]};
    // eager launches on the context's stream (no graph to instantiate, no timing events)
    const bool timing = c->timing;
    c->timing = false;
    s = enqueue_eval(c, c->stream, d_probs, d_err_bound, b);
    c->timing = timing;
    if (s != CGD_OK) return s;
    HIP_OK(hipMemcpyAsync(c->h_status, c->d_status, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipEventRecord(c->ev_status, c->stream));
    c->status_pending = true;
    c->last_static = true;
    return CGD_OK;
}

cgd_status cgd_grid_values(cgd_ctx *c, double *d_logg) {
    if (!c || !d_logg) return fail(CGD_ERR_ARG, "NULL argument");
    if (!c->evaluated || c->last_static) return fail(CGD_ERR_STATE, "cgd_grid_values needs a preceding cgd_eval");
    HIP_OK(hipMemcpyAsync(d_logg, c->d_logg, sizeof(double2) * c->npts, hipMemcpyDeviceToDevice, c->stream));
    return CGD_OK;
}

cgd_status cgd_grad(cgd_ctx *c, const double *d_dprobs, double *d_dr, double *d_dT, double *d_dalpha,
                    double *d_dschmidt) {
    if (!c) return fail(CGD_ERR_ARG, "ctx is NULL");
    if (!(c->flags & CGD_FLAG_GRAD)) return fail(CGD_ERR_STATE, "context created without CGD_FLAG_GRAD");
    if (!c->evaluated || c->last_static) return fail(CGD_ERR_STATE, "cgd_grad needs a preceding cgd_eval");
    if (!d_dprobs) return fail(CGD_ERR_ARG, "d_dprobs is NULL");
    cgd_status s = check_status(c);
    if (s != CGD_OK) return s;
    hipStream_t st = c->stream;
    // adjoint DFT: Ghat_k = (1/prod G) sum_b dL/dP(b) w_k^-b on the half grid
    HIP_OK(launch_adjoint_seed(c->d_inst, c->d_prob_prefix, c->n_inst, c->nprobs, d_dprobs, c->d_adj_off,
                               c->d_adjA, st));
    for (size_t si = 0; si < c->adj_stages.size(); ++si) {
        DftStage &S = c->adj_stages[si];
        const double2 *in = (si % 2 == 0) ? c->d_adjA : c->d_adjB;
        double2 *out = (si % 2 == 0) ? c->d_adjB : c->d_adjA;
        HIP_OK(launch_dft_stage(S.d_desc, S.d_prefix, (int)S.desc.size(), S.total, c->d_tw, in, out, nullptr,
                                nullptr, c->d_status, st));
    }
    HIP_OK(launch_adjoint_gather(c->d_inst, c->d_inst_pt_prefix, c->n_inst, c->npts, c->d_adj_off, c->d_adjA,
                                 c->d_adjB, c->d_ghat, st));
    // per (block, chunk of points): Gauss-Jordan inverse and accumulation
    for (auto &g : c->gadj) {
        if (g.jobs.empty()) continue;
        int nitems = 0;
        for (int32_t bj : g.jobs) nitems += c->gblocks[bj].nchunks;
        // job prefix holds absolute item indices; the launch covers this class's items
        AdjArgs a{g.d_jobs, g.d_prefix, (int)g.jobs.size(), c->adj_chunk, c->d_gblocks, c->d_inst, c->d_gpool,
                  c->d_grb, c->d_logg, c->d_ghat, c->d_partial, c->part_stride, 0, c->d_adj_work, c->adj_ldw,
                  c->adj_nwg};
        HIP_OK(launch_adjoint(g.cls, a, nitems, g.prefix[0], st));
    }
    HIP_OK(launch_adjoint_reduce(c->d_gblocks, c->d_z_prefix, (int)c->gblocks.size(), c->z_total, c->d_partial,
                                 c->part_stride, c->d_z, st));
    std::vector<cplx> zh(c->z_total);
    HIP_OK(hipMemcpyAsync(zh.data(), c->d_z, sizeof(double2) * c->z_total, hipMemcpyDeviceToHost, st));
    if (st) HIP_OK(hipStreamSynchronize(st)); else HIP_OK(hipDeviceSynchronize());
    // chain rule on the host (FP64), then upload
    std::vector<int64_t> roff(c->n_inst + 1, 0), toff(c->n_inst + 1, 0), soff(c->n_inst + 1, 0);
    for (int i = 0; i < c->n_inst; ++i) {
        const int M = c->hinst_copy[i].M;
        roff[i + 1] = roff[i] + M;
        toff[i + 1] = toff[i] + (int64_t)M * M;
        soff[i + 1] = soff[i] + c->hinst_copy[i].K;
    }
    std::vector<double> gr(roff[c->n_inst], 0.0), gs(soff[c->n_inst], 0.0);
    std::vector<cplx> gT(toff[c->n_inst], cplx(0, 0)), ga(roff[c->n_inst], cplx(0, 0));
    chain_rule(c, zh, gr, gT, ga, gs, roff, toff, soff);
    if (d_dr) HIP_OK(hipMemcpyAsync(d_dr, gr.data(), sizeof(double) * gr.size(), hipMemcpyHostToDevice, st));
    if (d_dT) HIP_OK(hipMemcpyAsync(d_dT, gT.data(), sizeof(cplx) * gT.size(), hipMemcpyHostToDevice, st));
    if (d_dalpha) HIP_OK(hipMemcpyAsync(d_dalpha, ga.data(), sizeof(cplx) * ga.size(), hipMemcpyHostToDevice, st));
    if (d_dschmidt)
        HIP_OK(hipMemcpyAsync(d_dschmidt, gs.data(), sizeof(double) * gs.size(), hipMemcpyHostToDevice, st));
    if (st) HIP_OK(hipStreamSynchronize(st)); else HIP_OK(hipDeviceSynchronize());
    return check_status(c);
}

cgd_status cgd_set_timing(cgd_ctx *c, int32_t enable) {
    if (!c) return fail(CGD_ERR_ARG, "ctx is NULL");
    c->timing = enable != 0;
    return CGD_OK;
}

cgd_status cgd_stage_times(cgd_ctx *c, double *ms) {
    if (!c || !ms) return fail(CGD_ERR_ARG, "NULL argument");
    if (!c->evaluated) return fail(CGD_ERR_STATE, "no evaluation yet");
    for (int i = 0; i < CGD_NSTAGES; ++i) ms[i] = -1.0;
    if (!c->timing) return CGD_OK;
    for (size_t k = 0; k < c->tev_stage.size(); ++k) {
        HIP_OK(hipEventSynchronize(c->tev[2 * k + 1]));
        float t = 0;
        HIP_OK(hipEventElapsedTime(&t, c->tev[2 * k], c->tev[2 * k + 1]));
        double &m = ms[c->tev_stage[k]];
        m = (m < 0 ? 0.0 : m) + t;
    }
    return CGD_OK;
}

cgd_status cgd_mixed_stats(cgd_ctx *c, int64_t *n_refactored, int64_t *n_total) {
    if (!c) return fail(CGD_ERR_ARG, "ctx is NULL");
    if (c->prec != CGD_PREC_MIXED || !c->evaluated || c->last_static)
        return fail(CGD_ERR_STATE, "cgd_mixed_stats needs a preceding mixed cgd_eval");
    int h[kG64];
    if (c->stream) HIP_OK(hipStreamSynchronize(c->stream)); else HIP_OK(hipDeviceSynchronize());
    HIP_OK(hipMemcpy(h, c->d_counts, sizeof(h), hipMemcpyDeviceToHost));
    int64_t tot = 0, all = 0;
    for (int k = 0; k < kG64; ++k) {
        tot += h[k];
        all += c->g64[k].nitems;
    }
    all += c->g64one.nitems;
    for (int k = 0; k < kMfmaClasses; ++k) all += c->g32[k].nitems;
    if (n_refactored) *n_refactored = tot;
    if (n_total) *n_total = all;
    return CGD_OK;
}

cgd_status cgd_stage_work(const cgd_ctx *c, double *flops, double *bytes) {
    if (!c) return fail(CGD_ERR_ARG, "ctx is NULL");
    for (int i = 0; i < CGD_NSTAGES; ++i) {
        if (flops) flops[i] = c->work_flops[i];
        if (bytes) bytes[i] = c->work_bytes[i];
    }
    return CGD_OK;
}

cgd_status cgd_bounds(const cgd_ctx *c, int32_t *grid, double *wrap_bound) {
    if (!c) return fail(CGD_ERR_ARG, "ctx is NULL");
    if (grid) std::copy(c->grid_used.begin(), c->grid_used.end(), grid);
    if (wrap_bound) std::copy(c->wrap_bound.begin(), c->wrap_bound.end(), wrap_bound);
    return CGD_OK;
}

cgd_status cgd_set_kernel_shape(cgd_ctx *c, int32_t size_class, int32_t fp64_shape, int32_t fp32_shape) {
    if (!c) return fail(CGD_ERR_ARG, "ctx is NULL");
    if (size_class < 0 || size_class >= kRegClasses) return fail(CGD_ERR_ARG, "size class out of range");
    const int k = size_class;
    bool keeps = false, fp32 = false;
    for (size_t b = 0; b < c->blocks.size(); ++b) {
        const BlockDev &d = c->blocks[b];
        if (c->is_hess[b] || d.lowrank || d.cls != k) continue;
        keeps |= d.nkeep > 0;
        fp32 |= d.fp32 && mfma_class_of(d.nb) == k;
    }
    if (fp64_shape >= 0) {
        const int lim = keeps ? reg_kernel_variants(k) : reg_variants(k);
        if (fp64_shape >= lim)
            return fail(CGD_ERR_ARG, "fp64 shape out of range for this class" +
                                         std::string(keeps ? " (blocks with kept modes need a register-kernel shape)" : ""));
    }
    if (fp32_shape >= 0) {
        if (!fp32) return fail(CGD_ERR_ARG, "this class has no FP32 pass");
        if (fp32_shape >= mfma_variants(k)) return fail(CGD_ERR_ARG, "fp32 shape out of range for this class");
    }
    if (fp64_shape >= 0) c->reg_var[k] = fp64_shape;
    if (fp32_shape >= 0) c->mfma_var[k] = fp32_shape;
    if (c->gexec) {  // the captured launch sequence names the old kernels
        (void)hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
    }
    return CGD_OK;
}

const char *cgd_tuning(const cgd_ctx *ctx) {
    if (!ctx) {
        fail(CGD_ERR_ARG, "ctx is NULL");
        return nullptr;
    }
    return ctx->tune_json.c_str();
}

void cgd_destroy(cgd_ctx *ctx) {
    if (!ctx) return;
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream); else (void)hipDeviceSynchronize();
    free_ctx(ctx);
}

const char *cgd_last_error(void) { return g_err.c_str(); }

}  // extern "C"
