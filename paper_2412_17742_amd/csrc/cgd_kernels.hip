// HIP kernels for gfx950 (CDNA4): per-grid-point factorisations of
// S(w) = I - diag(d(w)) H (Eq. q_d), their log-determinants with the
// continuous square-root branch, the displacement exponent, and the inverse
// grid DFT.
//
// Branch rule.  H = X A = I - Sigma^-1 is Hermitian with spectrum in (-1, 1)
// for every physical state (Sigma - I/2 > 0, the uncertainty relation of
// Sec. II), so for |w_l| <= 1 the matrix S(t w) is accretive for all t in
// [0, 1]: Re <x, S x> >= (1 - ||H||) |x|^2.  Schur complements of accretive
// matrices are accretive, hence every pivot of the unpivoted LU of S(t w) has
// a positive real part; the pivots move continuously from 1 (at t = 0), so
// log det S = sum_i Log(pivot_i) with principal logarithms is the continuous
// branch, and sqrt(det S) = exp(log det S / 2).
//
// Displacement exponent.  E(w) = 1/2 gamma^T S^-1 D X gamma (Eq. q_d
// numerator).  The matrix is bordered by one extra row and column,
//     S' = [[S, D X gamma], [gamma^T, 1]],
// whose last unpivoted pivot is the Schur complement 1 - gamma^T S^-1 D X gamma
// = 1 - 2 E, so E comes out of the same elimination with no triangular solve.
// The host stores the border inside H (row -gamma^T, column -X gamma, factor 1).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

#include "cgd_internal.h"

namespace cgd {

// ---------------------------------------------------------------------------
// small complex helpers (double2 = (re, im))
// ---------------------------------------------------------------------------
__device__ __forceinline__ double2 cmk(double re, double im) { return make_double2(re, im); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return cmk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a - l * u
__device__ __forceinline__ double2 cfnms(double2 a, double2 l, double2 u) {
    a.x = fma(-l.x, u.x, a.x);
    a.x = fma(l.y, u.y, a.x);
    a.y = fma(-l.x, u.y, a.y);
    a.y = fma(-l.y, u.x, a.y);
    return a;
}
// a + l * u
__device__ __forceinline__ double2 cfma(double2 l, double2 u, double2 a) {
    a.x = fma(l.x, u.x, a.x);
    a.x = fma(-l.y, u.y, a.x);
    a.y = fma(l.x, u.y, a.y);
    a.y = fma(l.y, u.x, a.y);
    return a;
}
// a + conj(l) * u
__device__ __forceinline__ double2 cfma_conj(double2 l, double2 u, double2 a) {
    a.x = fma(l.x, u.x, a.x);
    a.x = fma(l.y, u.y, a.x);
    a.y = fma(l.x, u.y, a.y);
    a.y = fma(-l.y, u.x, a.y);
    return a;
}
__device__ __forceinline__ double2 cinv(double2 d) {
    const double s = 1.0 / (d.x * d.x + d.y * d.y);
    return cmk(d.x * s, -d.y * s);
}
// principal logarithm
__device__ __forceinline__ double2 clog(double2 d) {
    return cmk(0.5 * log(d.x * d.x + d.y * d.y), atan2(d.y, d.x));
}

// Sum over i = tid, tid + nt, ... of the principal logarithms of pivot i
// (i < nl) and of the eigenvalue factor 1 - w_A lambda_i (i < n_eig).  Where
// both factors of an index lie in the right half-plane their arguments add
// up to less than pi in modulus, so the logarithm of their product is the
// sum of the two logarithms: one log and one atan2 per index instead of two.
template <typename PV>
__device__ __forceinline__ double2 pivot_eig_logs(const PV *piv, int nl, const double *__restrict__ lam, int n_eig,
                                                  double2 wa, int tid, int nt) {
    double2 acc = cmk(0.0, 0.0);
    const int n = nl > n_eig ? nl : n_eig;
    for (int i = tid; i < n; i += nt) {
        double2 f = cmk(1.0, 0.0), g = cmk(1.0, 0.0);
        if (i < nl) f = cmk((double)piv[i].x, (double)piv[i].y);
        if (i < n_eig) g = cmk(1.0 - wa.x * lam[i], -wa.y * lam[i]);
        double2 lg;
        if (f.x > 0.0 && g.x > 0.0) {
            lg = clog(cmul(f, g));
        } else {
            const double2 a = clog(f), b = clog(g);
            lg = cmk(a.x + b.x, a.y + b.y);
        }
        acc.x += lg.x;
        acc.y += lg.y;
    }
    return acc;
}

// Value of w at grid index k of an axis of extent G: the root of unity
// exp(2 pi i k / G), or, on a circle of radius rho > 0 in t (moments mode),
// w = exp(t) with t = rho exp(2 pi i k / G).
__device__ __forceinline__ double2 grid_w(int k, int G, double rho) {
    double s, c;
    sincospi(2.0 * (double)k / (double)G, &s, &c);
    if (rho == 0.0) return cmk(c, s);
    double s2, c2;
    sincos(rho * s, &s2, &c2);
    const double m = exp(rho * c);
    return cmk(m * c2, m * s2);
}

// Grid coordinates of evaluated point p of instance I (half grid on axis 0)
// and the corresponding value of w.
// An instance has at most 2^31 grid points (checked at create), so the index
// arithmetic is 32-bit.
__device__ __forceinline__ int point_k(const InstDev &I, int64_t p, int l) {
    unsigned stride = 1;
    for (int m = I.L - 1; m > l; --m) stride *= (unsigned)I.G[m];
    unsigned k = (unsigned)p / stride;
    if (l > 0) k %= (unsigned)I.G[l];
    return (int)k;
}
// On the unit circle w is read from the twiddle table when one is given:
// exp(2 pi i k / G) is the conjugate of the stored exp(-2 pi i k / G).
__device__ __forceinline__ void point_w(const InstDev &I, int64_t p, int l, double2 &w,
                                        const double2 *__restrict__ tw = nullptr) {
    const int k = point_k(I, p, l);
    if (tw != nullptr && I.rho == 0.0) {
        const double2 t = tw[I.tw_off[l] + k];
        w = cmk(t.x, -t.y);
    } else {
        w = grid_w(k, I.G[l], I.rho);
    }
}

// Largest c with prefix[c] <= item (prefix[0] = 0, strictly usable entries n).
__device__ __forceinline__ int find_job(const int64_t *__restrict__ prefix, int n, int64_t item, int lo = 0) {
    int hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= item) lo = mid; else hi = mid - 1;
    }
    return lo;
}
// The same from a hint: hint[item / 64] is the job of item 64 (item / 64), so
// the answer is at most a few entries further; a short forward scan replaces
// the chain of dependent loads of the binary search (which takes over when
// the scan runs long).
__device__ __forceinline__ int find_job_hinted(const int64_t *__restrict__ prefix, int n, int64_t item,
                                               const int32_t *__restrict__ hint) {
    int j = hint[item >> 6];
    for (int step = 0; step < 4; ++step) {
        if (j + 1 >= n || prefix[j + 1] > item) return j;
        ++j;
    }
    return find_job(prefix, n, item, j);
}

// Block-wide sum of a complex value over NT threads (deterministic order).
template <int NT>
__device__ __forceinline__ double2 block_sum(double2 v, double2 *s_red) {
    #pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        v.x += __shfl_xor(v.x, off, 64);
        v.y += __shfl_xor(v.y, off, 64);
    }
    constexpr int NW = (NT + 63) / 64;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (NW > 1) {
        if (lane == 0) s_red[wid] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            double2 t = s_red[0];
            for (int i = 1; i < NW; ++i) { t.x += s_red[i].x; t.y += s_red[i].y; }
            v = t;
        }
    }
    return v;  // valid in thread 0
}

// ---------------------------------------------------------------------------
// Kernel A: register-resident unpivoted LU, one workgroup per (block, point).
//
// The (padded) N x N matrix is distributed cyclically over a PR x PC thread
// grid: element (i, j) lives in thread (i % PR, j % PC) at register slot
// (i / PR, j / PC).  Step k broadcasts row k and column k through LDS
// (double-buffered, one barrier per step) and every thread applies the
// rank-1 update to its own elements.  The step loop is split into an
// unrolled loop over register rows r (k in [r PR, (r+1) PR)) so that every
// register index is a compile-time constant and the update only touches the
// register rows >= r and columns >= (r PR)/PC that can still be active.
//
// T = double: the FP64 path.  T = float: the first pass of the mixed path
// (matrix and elimination in complex FP32, logarithms of the pivots and
// their sum in FP64).  The workgroup loops over its items, either the
// contiguous range of a size class (job prefix sums) or an explicit list of
// (block, point) pairs built on the device.
// ---------------------------------------------------------------------------
template <typename T> struct cx2 { T x, y; };
template <typename T> __device__ __forceinline__ cx2<T> mk2(T a, T b) { cx2<T> r; r.x = a; r.y = b; return r; }
template <typename T> __device__ __forceinline__ cx2<T> mul2(cx2<T> a, cx2<T> b) {
    return mk2<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T> __device__ __forceinline__ cx2<T> fnms2(cx2<T> a, cx2<T> l, cx2<T> u) {
    a.x = fma(-l.x, u.x, a.x);
    a.x = fma(l.y, u.y, a.x);
    a.y = fma(-l.x, u.y, a.y);
    a.y = fma(-l.y, u.x, a.y);
    return a;
}
// 1/x from the hardware estimate and two Newton-Raphson steps
// y <- y + y (1 - x y) (the relative error squares at each step)
__device__ __forceinline__ double rcp_nr(double x) {
    double y = __builtin_amdgcn_rcp(x);
    y = fma(y, fma(-x, y, 1.0), y);
    return fma(y, fma(-x, y, 1.0), y);
}
__device__ __forceinline__ float rcp_nr(float x) { return __builtin_amdgcn_rcpf(x); }
template <typename T> __device__ __forceinline__ cx2<T> inv2(cx2<T> d) {
    const T s = rcp_nr(d.x * d.x + d.y * d.y);
    return mk2<T>(d.x * s, -d.y * s);
}
template <typename T> struct PoolT;
template <> struct PoolT<double> { typedef double2 type; };
template <> struct PoolT<float> { typedef float2 type; };

// Raw buffer view of one block's nb x nb matrix (row-major).  The buffer's own
// range check returns zero for every offset past its end, so padding rows and
// columns are read with no clamped addresses or selects: an element's offset
// is row_off + col_off, and either part is kPastEnd outside the matrix (the
// sum then lies past the end and below 2^31).
constexpr unsigned kPastEnd = 0x40000000u;
constexpr int kRawBufferWord3 = 0x00020000;  // untyped raw buffer, gfx9 family
template <typename PT> struct MatrixBuf {
    __amdgpu_buffer_rsrc_t r;
    int nb;
    __device__ __forceinline__ MatrixBuf(const PT *p, int n)
        : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(static_cast<const void *>(p)), (short)0,
                                              n * n * (int)sizeof(PT), kRawBufferWord3)),
          nb(n) {}
    __device__ __forceinline__ unsigned row_off(int i) const {
        return i < nb ? (unsigned)(i * nb) * (unsigned)sizeof(PT) : kPastEnd;
    }
    __device__ __forceinline__ unsigned col_off(int j) const {
        return j < nb ? (unsigned)j * (unsigned)sizeof(PT) : kPastEnd;
    }
    __device__ __forceinline__ PT load(unsigned off) const;
};
// The loaded vector is reinterpreted as a whole: with one bit cast per 32-bit
// element, this compiler narrows the b64 load to a single dword and returns
// it for both components.
typedef float f32x2v __attribute__((ext_vector_type(2)));
typedef double f64x2v __attribute__((ext_vector_type(2)));
template <> __device__ __forceinline__ float2 MatrixBuf<float2>::load(unsigned off) const {
    const f32x2v v = __builtin_bit_cast(f32x2v, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
    return make_float2(v.x, v.y);
}
template <> __device__ __forceinline__ double2 MatrixBuf<double2>::load(unsigned off) const {
    const f64x2v v = __builtin_bit_cast(f64x2v, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0));
    return make_double2(v.x, v.y);
}

struct LuArgs {
    const int32_t *job_block;
    const int64_t *job_prefix;
    int njobs;
    int64_t nitems;
    const int2 *list;         // explicit (block, point) items, or nullptr
    const int *list_count;
    const BlockDev *blocks;
    const InstDev *insts;
    const void *pool;         // double2 (FP64) or float2 (FP32) matrices
    const int32_t *rbpool;
    const double *eigpool;
    double2 *contrib;
    int *status;
    double2 *tpool;           // density mode: trailing Schur complements (nkeep + bordered)^2 per point
    const double2 *tw;        // twiddle table (roots of unity read instead of computed), or nullptr
    const int32_t *job_hint;  // job of item 64 c, per c (range launches), or nullptr
};

template <typename T, int PR, int PC, int TR, int TC>
__global__ void __launch_bounds__(PR *PC) lu_reg(const LuArgs A)
{
    typedef cx2<T> C;
    typedef typename PoolT<T>::type PT;
    constexpr int NT = PR * PC;
    constexpr int N = PR * TR;
    static_assert(PR * TR == PC * TC, "square padding");
    static_assert(PC % PR == 0, "column owner must be uniform over a register row");
    __shared__ C s_u[2][N];
    __shared__ C s_l[2][N];
    __shared__ C s_inv[2];
    __shared__ C s_d[N];
    __shared__ C s_piv[N];
    __shared__ double2 s_w[kMaxBins];
    __shared__ double2 s_red[NT / 64 + 1];
    __shared__ int s_bad;

    const int tid = threadIdx.x;
    const int tx = tid % PC, ty = tid / PC;
    {
        const int64_t item = blockIdx.x;
        if (A.list && item >= (int64_t)*A.list_count) return;
        int bi;
        int64_t pt;
        if (A.list) {
            const int2 e = A.list[item];
            bi = e.x;
            pt = e.y;
        } else {
            const int job = A.job_hint ? find_job_hinted(A.job_prefix, A.njobs, item, A.job_hint)
                                      : find_job(A.job_prefix, A.njobs, item);
            bi = A.job_block[job];
            pt = item - A.job_prefix[job];
        }
        const BlockDev B = A.blocks[bi];
        const InstDev &I = A.insts[B.inst];
        const int nb = B.nb;
        // pivots of S; a density-mode block stops there and keeps the trailing
        // (kept-mode and displacement) border as its Schur complement
        const int nS = nb - B.bordered - B.nkeep;
        const int nstop = B.nkeep ? nS : nb;

        if (tid < I.L) point_w(I, pt, tid, s_w[tid], A.tw);
        if (tid == 0) s_bad = 0;
        __syncthreads();
        // s_d = -d on the matrix rows, 0 on the padding: S = I + (-D) H
        for (int i = tid; i < N; i += NT) {
            C nd = mk2<T>(T(0), T(0));
            if (i < nb) {
                const int b = A.rbpool[B.rb_off + i];
                nd = b < 0 ? mk2<T>(T(-1), T(0)) : mk2<T>(-(T)s_w[b].x, -(T)s_w[b].y);
            }
            s_d[i] = nd;
        }
        __syncthreads();

        const PT *__restrict__ Hs = (const PT *)A.pool + B.h_off;
        if (B.hs_stride) Hs += (int64_t)point_k(I, pt, B.schur_axis) * B.hs_stride;
        const MatrixBuf<PT> hm(Hs, nb);

        C a[TR][TC];
        unsigned coff[TC];
        #pragma unroll
        for (int c = 0; c < TC; ++c) coff[c] = hm.col_off(c * PC + tx);
        #pragma unroll
        for (int r = 0; r < TR; ++r) {
            const int i = r * PR + ty;
            const unsigned roff = hm.row_off(i);
            const C nd = s_d[i];
            #pragma unroll
            for (int c = 0; c < TC; ++c) {
                const PT h = hm.load(roff + coff[c]);  // zero outside the matrix
                C v;
                v.x = fma(nd.x, h.x, -(nd.y * h.y));
                v.y = fma(nd.x, h.y, nd.y * h.x);
                if (i == c * PC + tx) v.x += T(1);
                a[r][c] = v;
            }
        }

        #pragma unroll
        for (int r = 0; r < TR; ++r) {
            const int cown = (r * PR) / PC;
            int kend = nstop - r * PR;
            kend = kend < 0 ? 0 : (kend > PR ? PR : kend);
            for (int kk = 0; kk < kend; ++kk) {
                const int k = r * PR + kk;
                const int buf = k & 1;
                if (ty == kk) {
                    #pragma unroll
                    for (int c = cown; c < TC; ++c) {
                        const int j = c * PC + tx;
                        if (j >= k) s_u[buf][j] = a[r][c];
                        if (j == k) {
                            // the pivot's owner publishes its reciprocal and records it
                            s_inv[buf] = inv2<T>(a[r][c]);
                            const C d = a[r][c];
                            s_piv[k] = d;
                            // pivots of S lie in the right half-plane; the border's (1 - 2E) need not
                            if (!isfinite(d.x) || !isfinite(d.y) || (k < nS && !(d.x > T(0)))) s_bad = 1;
                        }
                    }
                }
                if (tx == k % PC) {
                    #pragma unroll
                    for (int r2 = r; r2 < TR; ++r2) {
                        const int i = r2 * PR + ty;
                        if (i > k) s_l[buf][i] = a[r2][cown];
                    }
                }
                __syncthreads();
                const C dinv = s_inv[buf];
                C u[TC];
                #pragma unroll
                for (int c = cown; c < TC; ++c) {
                    const int j = c * PC + tx;
                    u[c] = (j > k && j < nb) ? s_u[buf][j] : mk2<T>(T(0), T(0));
                }
                #pragma unroll
                for (int r2 = r; r2 < TR; ++r2) {
                    const int i = r2 * PR + ty;
                    const C l = (i > k && i < nb) ? mul2<T>(s_l[buf][i], dinv) : mk2<T>(T(0), T(0));
                    #pragma unroll
                    for (int c = cown; c < TC; ++c) a[r2][c] = fnms2<T>(a[r2][c], l, u[c]);
                }
            }
        }
        __syncthreads();
        if (B.nkeep) {
            // density mode: the trailing (nkeep + bordered)^2 Schur complement, each
            // thread from its own registers
            const int nt = nb - nS;
            double2 *__restrict__ Tout = A.tpool + B.t_off + pt * (int64_t)(nt * nt);
            #pragma unroll
            for (int r = 0; r < TR; ++r) {
                const int i = r * PR + ty;
                #pragma unroll
                for (int c = 0; c < TC; ++c) {
                    const int j = c * PC + tx;
                    if (i >= nS && j >= nS && i < nb && j < nb)
                        Tout[(i - nS) * nt + (j - nS)] = cmk((double)a[r][c].x, (double)a[r][c].y);
                }
            }
        }

        // epilogue: -1/2 [sum_i Log(pivot_i) + sum_i Log(1 - w_A lambda_i)] + E, in FP64
        const int nlog = nS;
        double2 acc = pivot_eig_logs(s_piv, nlog, A.eigpool + B.eig_off, B.n_eig,
                                     B.n_eig > 0 ? s_w[B.schur_axis] : cmk(0.0, 0.0), tid, NT);
        acc = block_sum<NT>(acc, s_red);
        if (tid == 0) {
            double2 res = cmk(-0.5 * acc.x, -0.5 * acc.y);
            if (B.bordered && !B.nkeep) {
                const C p = s_piv[nb - 1];
                res.x += 0.5 * (1.0 - (double)p.x);
                res.y += 0.5 * (0.0 - (double)p.y);
            }
            A.contrib[I.c_off + pt * I.nblocks + B.blk] = res;
            if (s_bad) atomicOr(A.status, 1);
        }
    }
}

// ---------------------------------------------------------------------------
// Kernel M: complex FP32 unpivoted LU on MFMA (first pass of the mixed path).
//
// The padded 16 NTILE x 16 NTILE matrix is split into 16 x 16 tiles; tile
// (I, J) is held by wave (I mod WR, J mod WC) as two MFMA accumulators (real
// and imaginary part) in the 16x16x4 f32 layout: lane l, register v holds
// element (4 (l/16) + v, l mod 16) of the tile.  Elimination goes one tile
// column at a time.  With D the diagonal tile, X the tiles below it and Y the
// tiles to its right (all after the previous steps), the trailing matrix takes
// the Schur complement update
//     A22 <- A22 - X W,    W = D^-1 Y,
// as 16 MFMAs per tile (K = 16, complex product as four real products).
// det S is the product of det D over the steps, and the pivots of D's own
// unpivoted elimination are the pivots of S.  One step J:
//   1. every wave updates its tiles, those of tile row and column J+1 first;
//      the owner of tile (J+1, J+1) then inverts it by Gauss-Jordan elimination in registers (row
//      broadcast by lane-swap permutes, column broadcast by DPP
//      row_newbcast), recording its pivots, while the other waves carry on
//      with the rest of the update;
//   2. barrier; the owners of tile column J+1 write X (negated, transposed)
//      to LDS and the owners of tile row J+1 form W = D^-1 Y on MFMA from
//      their own accumulators and write it to LDS; barrier.
// Every LDS panel is read only before the barrier that precedes its next
// write, so each has one buffer; Y stays in its owner's accumulators (W is
// formed by the wave that holds the tile).  Order 64: 19.4 KB per workgroup,
// eight workgroups per CU.  OCC > 1 caps the registers so that OCC waves fit per
// SIMD (the autotuner times both).  Padding rows and columns hold
// the identity and stay decoupled, so they add pivots equal to 1.  The
// epilogue (FP64) is the same as in the register kernel.
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// Element-type traits of the MFMA LU: FP32 uses v_mfma_f32_16x16x4f32, whose
// accumulator holds element (4g + v, c) in lane (g, c) = (l / 16, l % 16),
// register v; FP64 uses v_mfma_f64_16x16x4f64, whose accumulator holds
// element (g + 4v, c).  Both take A[i][k] from lane (k, i) and B[k][j] from
// lane (k, j).
template <typename T> struct MfmaT;
template <> struct MfmaT<float> {
    typedef f32x4 V4;
    __device__ static __forceinline__ V4 mfma(float a, float b, V4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ int row(int g, int v) { return 4 * g + v; }
    __device__ static __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
};
template <> struct MfmaT<double> {
    typedef f64x4 V4;
    __device__ static __forceinline__ V4 mfma(double a, double b, V4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ int row(int g, int v) { return g + 4 * v; }
    __device__ static __forceinline__ double rcp(double x) { return rcp_nr(x); }
};

__device__ __forceinline__ float2 f2(float x, float y) { return make_float2(x, y); }

// Cross-lane moves on 32-bit registers; the FP64 forms move both halves.
template <int K> __device__ __forceinline__ unsigned dpp_row_bcast(unsigned x) {
    return (unsigned)__builtin_amdgcn_mov_dpp((int)x, 0x150 + K, 0xf, 0xf, true);
}
template <int K>
__device__ __forceinline__ float row_bcast(float x) {  // lane K of each 16-lane row to the whole row
    return __builtin_bit_cast(float, dpp_row_bcast<K>(__builtin_bit_cast(unsigned, x)));
}
template <int K>
__device__ __forceinline__ double row_bcast(double x) {  // one 64-bit DPP move (row_newbcast)
    return __builtin_amdgcn_update_dpp(0.0, x, 0x150 + K, 0xf, 0xf, true);
}

// 16-lane row G of a pair of registers (x, y) to all four rows of both (lane
// c of every row reads lane 16 G + c) through ds_bpermute: one LDS-pipe
// instruction per 32 bits, off the VALU (three lane swaps and their register
// copies did the same on the VALU at 172 more VALU instructions per wave).
template <int G> __device__ __forceinline__ unsigned group_bcast_u(unsigned x, int c) {
    return (unsigned)__builtin_amdgcn_ds_bpermute((G * 16 + c) * 4, (int)x);
}
template <int G>
__device__ __forceinline__ void group_bcast_pair(float x, float y, int c, float &ox, float &oy) {
    ox = __builtin_bit_cast(float, group_bcast_u<G>(__builtin_bit_cast(unsigned, x), c));
    oy = __builtin_bit_cast(float, group_bcast_u<G>(__builtin_bit_cast(unsigned, y), c));
}
template <int G>
__device__ __forceinline__ void group_bcast_pair(double x, double y, int c, double &ox, double &oy) {
    const uint2 u = __builtin_bit_cast(uint2, x), v = __builtin_bit_cast(uint2, y);
    ox = __builtin_bit_cast(double, make_uint2(group_bcast_u<G>(u.x, c), group_bcast_u<G>(u.y, c)));
    oy = __builtin_bit_cast(double, make_uint2(group_bcast_u<G>(v.x, c), group_bcast_u<G>(v.y, c)));
}

// 4 x 4 transpose between the lane group (lane / 16) and the register index:
// out[s] in lane group g is in[g] of lane group s, same lane within the group.
// v_permlane32_swap exchanges groups (2, 3) of its first operand with groups
// (0, 1) of its second, v_permlane16_swap groups (1, 3) of the first with
// (0, 2) of the second: two stages of two swaps (VALU only).  Needed for the
// FP32 layout only (FP64 accumulators are already in the B-operand layout).
__device__ __forceinline__ void swap32(float a, float b, float &na, float &nb) {
    const auto h = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(unsigned, a), __builtin_bit_cast(unsigned, b),
                                                    false, false);
    na = __builtin_bit_cast(float, (unsigned)h[0]);
    nb = __builtin_bit_cast(float, (unsigned)h[1]);
}
__device__ __forceinline__ void swap16(float a, float b, float &na, float &nb) {
    const auto h = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(unsigned, a), __builtin_bit_cast(unsigned, b),
                                                    false, false);
    na = __builtin_bit_cast(float, (unsigned)h[0]);
    nb = __builtin_bit_cast(float, (unsigned)h[1]);
}
__device__ __forceinline__ void group_reg_transpose(const f32x4 &in, float (&out)[4]) {
    float a0, a1, a2, a3;
    swap32(in[0], in[2], a0, a2);  // a0 = (in0[0], in0[1], in2[0], in2[1]), a2 = (in0[2], in0[3], in2[2], in2[3])
    swap32(in[1], in[3], a1, a3);
    swap16(a0, a1, out[0], out[1]);  // out0 = (in0[0], in1[0], in2[0], in3[0]), out1 = (.. [1])
    swap16(a2, a3, out[2], out[3]);
}

// old with lane L replaced by the wave-uniform x: one v_writelane per 32 bits
// with an immediate lane (the builtin form is turned into a select on a lane
// mask, which costs a mask per lane kept in registers)
template <int L> __device__ __forceinline__ unsigned write_lane_u(unsigned old, unsigned x) {
    unsigned r;
    asm("v_writelane_b32 %0, %1, %2" : "=v"(r) : "s"(x), "i"(L), "0"(old));
    return r;
}
template <int L> __device__ __forceinline__ float write_lane(float old, float x) {
    return __builtin_bit_cast(float, write_lane_u<L>(__builtin_bit_cast(unsigned, old), __builtin_bit_cast(unsigned, x)));
}
template <int L> __device__ __forceinline__ double write_lane(double old, double x) {
    const uint2 o = __builtin_bit_cast(uint2, old), u = __builtin_bit_cast(uint2, x);
    return __builtin_bit_cast(double, make_uint2(write_lane_u<L>(o.x, u.x), write_lane_u<L>(o.y, u.y)));
}

__device__ __forceinline__ float uniform_read(float x, int src_lane) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), src_lane));
}
__device__ __forceinline__ double uniform_read(double x, int src_lane) {
    const uint2 u = __builtin_bit_cast(uint2, x);
    return __builtin_bit_cast(double, make_uint2((unsigned)__builtin_amdgcn_readlane((int)u.x, src_lane),
                                                 (unsigned)__builtin_amdgcn_readlane((int)u.y, src_lane)));
}

// Gauss-Jordan inversion of a 16 x 16 tile held as lane (g, c), register v:
// element (4g + v, c) (both element types; the FP64 kernel stages its tile
// through LDS into this layout).  Step k, with p = a[k][k]:
// a[k][c] <- a[k][c]/p, a[r][k] <- -a[r][k]/p, a[k][k] <- 1/p and
// a[r][c] <- a[r][c] - a[r][k] a[k][c]/p elsewhere.  After the 16 steps the
// tile holds its inverse; p is the k-th pivot of the unpivoted LU.  Row k
// reaches every lane group by ds_bpermute and column k every lane of its row
// by DPP row_newbcast; each step updates row k+1 first, so that its broadcast
// overlaps the rest of the step.
template <int K, typename T>
__device__ __forceinline__ void gj_step(T (&ar)[4], T (&ai)[4], int g, int c, T &rowr, T &rowi, T &pr, T &pi) {
    constexpr int KG = K >> 2, KV = K & 3;
    constexpr int V1 = (K + 1) & 3, G1 = (K + 1) >> 2;
    T colr[4], coli[4];
    #pragma unroll
    for (int v = 0; v < 4; ++v) {
        colr[v] = row_bcast<K>(ar[v]);
        coli[v] = row_bcast<K>(ai[v]);
    }
    const T s = MfmaT<T>::rcp(pr * pr + pi * pi);
    const T rpr = pr * s, rpi = -pi * s;
    // t = a[k][c] / p off column k.  On column k, t = 1 + 1/p, so that the
    // common update a - a[r][k] t leaves -a[r][k] / p there with no zeroing of
    // a (|1/p| > 1/2 for an accretive matrix, so nothing cancels badly).
    const bool isk = (c == K);
    const T tr = isk ? T(1) + rpr : fma(rowr, rpr, -rowi * rpi);
    const T ti = isk ? rpi : fma(rowr, rpi, rowi * rpr);
    auto upd = [&](int v) {
        ar[v] = fma(coli[v], ti, fma(-colr[v], tr, ar[v]));
        ai[v] = fma(-coli[v], tr, fma(-colr[v], ti, ai[v]));
    };
    if (K < 15) {
        upd(V1);  // row K+1 (on group G1) first
        group_bcast_pair<G1>(ar[V1], ai[V1], c, rowr, rowi);
        pr = uniform_read(ar[V1], G1 * 16 + K + 1);
        pi = uniform_read(ai[V1], G1 * 16 + K + 1);
    }
    #pragma unroll
    for (int v = 0; v < 4; ++v)
        if (K == 15 || v != V1) upd(v);
    if (g == KG) {  // row k: a[k][c] / p, and 1/p at (k, k)
        ar[KV] = isk ? rpr : tr;
        ai[KV] = ti;
    }
}

// Runs steps 0 .. kstop - 1 (kstop wave-uniform); pivot k ends up in lane k
// of (pvr, pvi).  With kstop < 16 the tile is not inverted, but its first
// kstop pivots are exact: the last tile of a matrix needs only its pivots,
// and its rows and columns past the matrix are decoupled identity.
template <typename T, int... K>
__device__ __forceinline__ void gj_all(T (&ar)[4], T (&ai)[4], int g, int c, T &pvr, T &pvi, int kstop,
                                       std::integer_sequence<int, K...>) {
    T rowr, rowi;
    group_bcast_pair<0>(ar[0], ai[0], c, rowr, rowi);
    T pr = uniform_read(ar[0], 0), pi = uniform_read(ai[0], 0);
    pvr = pr;
    pvi = pi;
    // pivot k (wave-uniform after its step) into lane k
    auto keep = [&](auto kc) {
        constexpr int k = decltype(kc)::value;
        if constexpr (k < 16) {
            pvr = write_lane<k>(pvr, pr);
            pvi = write_lane<k>(pvi, pi);
        }
    };
    ((K < kstop ? (gj_step<K>(ar, ai, g, c, rowr, rowi, pr, pi), keep(std::integral_constant<int, K + 1>{}))
                : void()), ...);
}

template <typename T, int NTILE, int WR, int WC>
struct MfmaLds {
    typedef cx2<T> C;
    static constexpr int N = 16 * NTILE;
    // The panels hold tile rows (X) and tile columns (W) 1 .. NTILE - 1 only:
    // tile 0 is never below or right of a diagonal tile (one tile: no panels,
    // a placeholder column).
    static constexpr int NP = NTILE > 1 ? N - 16 : 1;  // panel width
    static constexpr int XS = NP + 1;  // padded stride of the transposed X panel
    C XT[16][XS];                      // -X^T of the step's tile column, tile rows 1 ..
    C W[16][NP];                       // W = D^-1 Y, tile columns 1 ..
    C DiT[16][17];                    // (D^-1)^T
    C d[N];
    C piv[N];
    double2 w[kMaxBins];
    double2 red[WR * WC + 1];
    int bad;
};

template <typename T, int NTILE, int WR, int WC>
__device__ __forceinline__ void lu_mfma_body(const LuArgs &A)
{
    typedef cx2<T> C;
    typedef typename PoolT<T>::type PT;
    typedef typename MfmaT<T>::V4 V4;
    constexpr bool F64 = sizeof(T) == 8;
    constexpr int NW = WR * WC;
    constexpr int NT = 64 * NW;
    constexpr int TRW = (NTILE + WR - 1) / WR;
    constexpr int TCW = (NTILE + WC - 1) / WC;
    using Lds = MfmaLds<T, NTILE, WR, WC>;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    Lds &S = *reinterpret_cast<Lds *>(lds_raw);

    const int tid = threadIdx.x;
    // the wave index as a scalar: every tile condition is a scalar branch
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int wr = wave / WC, wc = wave % WC;
    const int lg = lane >> 4, lc = lane & 15;

    const int64_t item = blockIdx.x;
    if (A.list && item >= (int64_t)*A.list_count) return;
    int bi;
    int64_t pt;
    if (A.list) {
        const int2 e = A.list[item];
        bi = e.x;
        pt = e.y;
    } else {
        const int job = A.job_hint ? find_job_hinted(A.job_prefix, A.njobs, item, A.job_hint)
                                      : find_job(A.job_prefix, A.njobs, item);
        bi = A.job_block[job];
        pt = item - A.job_prefix[job];
    }
    const BlockDev B = A.blocks[bi];
    const InstDev &I = A.insts[B.inst];
    const int nb = B.nb;
    const int nl = nb - B.bordered;  // pivots of S (the border's need not be in the right half-plane)
    const int ntl = (nb + 15) >> 4;  // tiles in use

    if (tid < I.L) point_w(I, pt, tid, S.w[tid], A.tw);
    if (tid == 0) S.bad = 0;
    __syncthreads();
    // S.d = -d on the matrix rows, 0 on the padding: S = I + (-D) H
    for (int i = tid; i < Lds::N; i += NT) {
        C nd = mk2<T>(T(0), T(0));
        if (i < nb) {
            const int b = A.rbpool[B.rb_off + i];
            nd = b < 0 ? mk2<T>(T(-1), T(0)) : mk2<T>(-(T)S.w[b].x, -(T)S.w[b].y);
        }
        S.d[i] = nd;
    }
    __syncthreads();

    const PT *__restrict__ Hs = (const PT *)A.pool + B.h_off;
    if (B.hs_stride) Hs += (int64_t)point_k(I, pt, B.schur_axis) * B.hs_stride;
    const MatrixBuf<PT> hm(Hs, nb);

    // Tile rows past the last tile in use stay zero (never read); in the
    // others, columns past the matrix read as zero from the buffer and the
    // diagonal tile adds the identity (padding included).
    V4 ar[TRW][TCW], ai[TRW][TCW];
    unsigned coff[TCW];
    #pragma unroll
    for (int tj = 0; tj < TCW; ++tj) coff[tj] = hm.col_off((wc + tj * WC) * 16 + lc);
    #pragma unroll
    for (int ti = 0; ti < TRW; ++ti) {
        const int It = wr + ti * WR;
        #pragma unroll
        for (int tj = 0; tj < TCW; ++tj) {
            ar[ti][tj] = V4{T(0), T(0), T(0), T(0)};
            ai[ti][tj] = V4{T(0), T(0), T(0), T(0)};
        }
        if (It >= ntl) continue;
        unsigned roff[4];
        C nd[4];
        #pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = It * 16 + MfmaT<T>::row(lg, v);
            roff[v] = hm.row_off(i);
            nd[v] = S.d[i];
        }
        #pragma unroll
        for (int tj = 0; tj < TCW; ++tj) {
            #pragma unroll
            for (int v = 0; v < 4; ++v) {
                const PT h = hm.load(roff[v] + coff[tj]);
                ar[ti][tj][v] = fma(nd[v].x, h.x, -(nd[v].y * h.y));
                ai[ti][tj][v] = fma(nd[v].x, h.y, nd[v].y * h.x);
            }
            if (It == wc + tj * WC) {
                #pragma unroll
                for (int v = 0; v < 4; ++v)
                    if (MfmaT<T>::row(lg, v) == lc) ar[ti][tj][v] += T(1);
            }
        }
    }

    // Publish what step Jn needs: -X^T (tiles below the diagonal), Y (tiles
    // right of it), and D^-1 with the pivots (diagonal tile).  Tiles are
    // addressed only with compile-time indices under wave-uniform branches (a
    // runtime-indexed copy of the accumulators would go through scratch); the
    // diagonal tile reaches the Gauss-Jordan registers through LDS.
    // -X^T of tile column Jn (after the barrier that ends the previous step's reads)
    auto publish_x = [&](int Jn) {
        const int stj = Jn / WC;
        if (wc != Jn % WC) return;
        #pragma unroll
        for (int ti = 0; ti < TRW; ++ti) {
            const int It = wr + ti * WR;
            #pragma unroll
            for (int tj = 0; tj < TCW; ++tj) {
                if (tj == stj && It > Jn && It < ntl) {
                    #pragma unroll
                    for (int v = 0; v < 4; ++v)
                        S.XT[lc][(It - 1) * 16 + MfmaT<T>::row(lg, v)] = mk2<T>(-ar[ti][tj][v], -ai[ti][tj][v]);
                }
            }
        }
    };
    auto publish = [&](int Jn) {
        const int sti = Jn / WR, stj = Jn / WC;
        const bool own_r = (wr == Jn % WR), own_c = (wc == Jn % WC);
        #pragma unroll
        for (int ti = 0; ti < TRW; ++ti) {
            #pragma unroll
            for (int tj = 0; tj < TCW; ++tj) {
                if (own_r && own_c && ti == sti && tj == stj) {
                    #pragma unroll
                    for (int v = 0; v < 4; ++v) S.DiT[MfmaT<T>::row(lg, v)][lc] = mk2<T>(ar[ti][tj][v], ai[ti][tj][v]);
                }
            }
        }
        if (own_r && own_c) {
            // the tile went to DiT untransposed; this wave alone reads it back
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            T gr[4], gi[4];
            #pragma unroll
            for (int v = 0; v < 4; ++v) {
                const C x = S.DiT[4 * lg + v][lc];
                gr[v] = x.x;
                gi[v] = x.y;
            }
            __builtin_amdgcn_wave_barrier();
            T pvr, pvi;
            // the last tile: only its pivots (no trailing tiles use its inverse)
            const int kstop = (Jn + 1 == ntl) ? nb - 16 * Jn : 16;
            gj_all(gr, gi, lg, lc, pvr, pvi, kstop, std::make_integer_sequence<int, 16>{});
            #pragma unroll
            for (int v = 0; v < 4; ++v) S.DiT[lc][4 * lg + v] = mk2<T>(gr[v], gi[v]);
            const int gk = Jn * 16 + lane;
            if (lane < 16 && gk < nb) {
                S.piv[gk] = mk2<T>(pvr, pvi);
                if (!isfinite(pvr) || !isfinite(pvi) || (gk < nl && !(pvr > T(0)))) S.bad = 1;
            }
        }
    };

    // W = D^-1 Y for this wave's tiles of tile row Jn (after the barrier that
    // publishes D^-1).
    // The B operand of chunk s at lane (g, c) is Y[4s + g][c], which the
    // owner holds in lane (s, c), register g: a lane-group/register
    // transpose of its accumulators (no LDS panel for Y).
    auto form_w = [&](int Jn) {
        if (wr != Jn % WR) return;
        const int sti = Jn / WR;
        T dr[4], di[4], dn[4];
        #pragma unroll
        for (int s = 0; s < 4; ++s) {
            const C x = S.DiT[4 * s + lg][lc];  // A operand: D^-1[l%16][4s + l/16]
            dr[s] = x.x;
            di[s] = x.y;
            dn[s] = -x.y;
        }
        #pragma unroll
        for (int tj = 0; tj < TCW; ++tj) {
            const int Jt = wc + tj * WC;
            if (Jt > Jn && Jt < ntl) {
                // B operand of chunk s: Y[4s + g][c]; in the FP64 layout that is
                // register s of the same lane, in the FP32 layout a transpose
                T yr[4] = {T(0), T(0), T(0), T(0)}, yi[4] = {T(0), T(0), T(0), T(0)};
                #pragma unroll
                for (int ti = 0; ti < TRW; ++ti)
                    if (ti == sti) {
                        if constexpr (F64) {
                            #pragma unroll
                            for (int s = 0; s < 4; ++s) {
                                yr[s] = ar[ti][tj][s];
                                yi[s] = ai[ti][tj][s];
                            }
                        } else {
                            group_reg_transpose(ar[ti][tj], yr);
                            group_reg_transpose(ai[ti][tj], yi);
                        }
                    }
                V4 wr_ = {T(0), T(0), T(0), T(0)}, wi_ = {T(0), T(0), T(0), T(0)};
                #pragma unroll
                for (int s = 0; s < 4; ++s) {
                    wr_ = MfmaT<T>::mfma(dr[s], yr[s], wr_);
                    wr_ = MfmaT<T>::mfma(dn[s], yi[s], wr_);
                    wi_ = MfmaT<T>::mfma(dr[s], yi[s], wi_);
                    wi_ = MfmaT<T>::mfma(di[s], yr[s], wi_);
                }
                #pragma unroll
                for (int v = 0; v < 4; ++v) S.W[MfmaT<T>::row(lg, v)][(Jt - 1) * 16 + lc] = mk2<T>(wr_[v], wi_[v]);
            }
        }
    };

    if (ntl > 0) {
        publish(0);
        __syncthreads();
        publish_x(0);
        form_w(0);
        __syncthreads();
    }

    #pragma unroll 1
    for (int J = 0; J + 1 < ntl; ++J) {
        const int Jn = J + 1;
        // A += (-X) W: real part (-Xr) Wr + Xi Wi, imaginary part (-Xr) Wi + (-Xi) Wr.
        // Operands from LDS: A = -X[row, 16J + 4s + l/16] per tile row, B =
        // W[4s + l/16, col] per pass (not held across the diagonal inversion).
        // The real part needs one negated operand (-Xi Wi): it is taken on
        // the W side when a wave holds fewer tile columns than tile rows, else
        // on the X side.  W is read only for the tile columns in use (the MFMA
        // loop below skips exactly the others).
        auto update = [&](int pass) {
            constexpr bool NEG_W = TCW < TRW;
            T wr_[TCW][4], wi_[TCW][4], wn_[TCW][4];
            #pragma unroll
            for (int tj = 0; tj < TCW; ++tj) {
                const int Jt = wc + tj * WC;
                if (Jt > J && Jt < ntl && (pass == 0 || Jt != Jn)) {
                    #pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        const C w = S.W[4 * s + lg][(Jt - 1) * 16 + lc];
                        wr_[tj][s] = w.x;
                        wi_[tj][s] = w.y;
                        if constexpr (NEG_W) wn_[tj][s] = -w.y;
                    }
                }
            }
            #pragma unroll
            for (int ti = 0; ti < TRW; ++ti) {
                const int It = wr + ti * WR;
                if (It <= J || It >= ntl) continue;
                if (pass == 1 && It == Jn) continue;  // tile row Jn went entirely in pass 0
                T xr[4], xi[4], xn[4];
                #pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const C x = S.XT[4 * s + lg][(It - 1) * 16 + lc];
                    xr[s] = x.x;
                    xi[s] = x.y;
                    if constexpr (!NEG_W) xn[s] = -x.y;
                }
                #pragma unroll
                for (int tj = 0; tj < TCW; ++tj) {
                    const int Jt = wc + tj * WC;
                    if (Jt <= J || Jt >= ntl) continue;
                    const bool first = (It == Jn) || (Jt == Jn);
                    if (first != (pass == 0)) continue;
                    #pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        ar[ti][tj] = MfmaT<T>::mfma(xr[s], wr_[tj][s], ar[ti][tj]);
                        ai[ti][tj] = MfmaT<T>::mfma(xr[s], wi_[tj][s], ai[ti][tj]);
                        if constexpr (NEG_W)
                            ar[ti][tj] = MfmaT<T>::mfma(xi[s], wn_[tj][s], ar[ti][tj]);
                        else
                            ar[ti][tj] = MfmaT<T>::mfma(xn[s], wi_[tj][s], ar[ti][tj]);
                        ai[ti][tj] = MfmaT<T>::mfma(xi[s], wr_[tj][s], ai[ti][tj]);
                    }
                }
            }
        };
        update(0);
        publish(Jn);
        update(1);
        __syncthreads();
        publish_x(Jn);
        form_w(Jn);
        __syncthreads();
    }

    double2 acc = pivot_eig_logs(S.piv, nl, A.eigpool + B.eig_off, B.n_eig,
                                 B.n_eig > 0 ? S.w[B.schur_axis] : cmk(0.0, 0.0), tid, NT);
    acc = block_sum<NT>(acc, S.red);
    if (tid == 0) {
        double2 res = cmk(-0.5 * acc.x, -0.5 * acc.y);
        if (B.bordered) {
            const C pb = S.piv[nb - 1];
            res.x += 0.5 * (1.0 - (double)pb.x);
            res.y += 0.5 * (0.0 - (double)pb.y);
        }
        A.contrib[I.c_off + pt * I.nblocks + B.blk] = res;
        if (S.bad) atomicOr(A.status, 1);
    }
}


template <int NTILE, int WR, int WC, int OCC = 1>
__global__ void __launch_bounds__(64 * WR * WC) __attribute__((amdgpu_waves_per_eu(OCC))) lu_mfma_f32(const LuArgs A)
{
    lu_mfma_body<float, NTILE, WR, WC>(A);
}

// The same elimination in complex FP64 on v_mfma_f64_16x16x4f64 (an FP64
// kernel shape the autotuner times against the register kernel).
template <int NTILE, int WR, int WC, int OCC = 1>
__global__ void __launch_bounds__(64 * WR * WC) __attribute__((amdgpu_waves_per_eu(OCC))) lu_mfma_f64(const LuArgs A)
{
    lu_mfma_body<double, NTILE, WR, WC>(A);
}

// ---------------------------------------------------------------------------
// Kernel B: unpivoted LU for orders above the register-resident limit.  One
// workgroup per (block, point), persistent over the work list; the matrix
// lives in a per-workgroup global workspace (L2/MALL resident) and is
// factorised right-looking in panels of kPanel columns: the panel is
// factorised in LDS, the U row block is solved in place, and the trailing
// matrix is updated in 64 x 64 tiles with 4 x 4 register blocks per thread
// against an LDS-staged U tile.
// ---------------------------------------------------------------------------
constexpr int kPanel = 16;
constexpr int kBigThreads = 256;

// Right-looking blocked unpivoted LU of W (order nb, leading dimension ldw,
// in global memory) for the pivots k < kstop, the steps of lu_big_f64: each
// panel of kPanel columns is factorised in LDS, the U row block is solved in
// place, and the trailing matrix (all rows and columns >= the panel's end) is
// updated in 64 x 64 tiles with 4 x 4 register blocks per thread against an
// LDS-staged U tile.  Pivots go to s_piv; *s_bad is set for a non-finite
// pivot, or one with Re <= 0 among the first check_lim.  With kstop < nb,
// W[kstop:, kstop:] ends as the Schur complement of the leading block.
__device__ __forceinline__ void big_lu_steps(double2 *__restrict__ W, int ldw, int nb, int kstop, int check_lim,
                                             double2 *s_panel, double2 *s_utile, double2 *s_piv, int *s_bad)
{
    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4;
    for (int k0 = 0; k0 < kstop; k0 += kPanel) {
        const int kb = min(kPanel, kstop - k0);
        const int mrows = nb - k0;
        // panel -> LDS
        for (int e = tid; e < mrows * kPanel; e += kBigThreads) {
            const int i = e / kPanel, t = e % kPanel;
            s_panel[e] = t < kb ? W[(size_t)(k0 + i) * ldw + k0 + t] : cmk(0.0, 0.0);
        }
        __syncthreads();
        for (int kk = 0; kk < kb; ++kk) {
            const double2 d = s_panel[kk * kPanel + kk];
            if (tid == 0) {
                s_piv[k0 + kk] = d;
                if (!isfinite(d.x) || !isfinite(d.y) || (k0 + kk < check_lim && !(d.x > 0.0))) *s_bad = 1;
            }
            const double2 dinv = cinv(d);
            for (int i = kk + 1 + tid; i < mrows; i += kBigThreads) {
                const double2 l = cmul(s_panel[i * kPanel + kk], dinv);
                s_panel[i * kPanel + kk] = l;
                for (int t = kk + 1; t < kb; ++t)
                    s_panel[i * kPanel + t] = cfnms(s_panel[i * kPanel + t], l, s_panel[kk * kPanel + t]);
            }
            __syncthreads();
        }
        const int j0 = k0 + kb;
        if (j0 >= nb) break;
        // U12 = L11^-1 A12 (unit lower triangular solve), in place in W
        for (int j = j0 + tid; j < nb; j += kBigThreads) {
            double2 x[kPanel];
            #pragma unroll
            for (int t = 0; t < kPanel; ++t) x[t] = t < kb ? W[(size_t)(k0 + t) * ldw + j] : cmk(0.0, 0.0);
            #pragma unroll
            for (int t = 1; t < kPanel; ++t) {
                #pragma unroll
                for (int s2 = 0; s2 < t; ++s2) x[t] = cfnms(x[t], s_panel[t * kPanel + s2], x[s2]);
            }
            #pragma unroll
            for (int t = 0; t < kPanel; ++t)
                if (t < kb) W[(size_t)(k0 + t) * ldw + j] = x[t];
        }
        __syncthreads();
        // trailing update A22 -= L21 U12
        for (int jt = j0; jt < nb; jt += 64) {
            for (int e = tid; e < kPanel * 64; e += kBigThreads) {
                const int t = e / 64, jj = jt + (e % 64);
                s_utile[e] = (t < kb && jj < nb) ? W[(size_t)(k0 + t) * ldw + jj] : cmk(0.0, 0.0);
            }
            __syncthreads();
            for (int it = j0; it < nb; it += 64) {
                double2 acc[4][4];
                #pragma unroll
                for (int a = 0; a < 4; ++a)
                    #pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        const int i = it + ty + 16 * a, j = jt + tx + 16 * b;
                        acc[a][b] = (i < nb && j < nb) ? W[(size_t)i * ldw + j] : cmk(0.0, 0.0);
                    }
                for (int t = 0; t < kb; ++t) {
                    double2 l[4], u[4];
                    #pragma unroll
                    for (int a = 0; a < 4; ++a) {
                        const int i = it + ty + 16 * a;
                        l[a] = i < nb ? s_panel[(i - k0) * kPanel + t] : cmk(0.0, 0.0);
                    }
                    #pragma unroll
                    for (int b = 0; b < 4; ++b) u[b] = s_utile[t * 64 + tx + 16 * b];
                    #pragma unroll
                    for (int a = 0; a < 4; ++a)
                        #pragma unroll
                        for (int b = 0; b < 4; ++b) acc[a][b] = cfnms(acc[a][b], l[a], u[b]);
                }
                #pragma unroll
                for (int a = 0; a < 4; ++a)
                    #pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        const int i = it + ty + 16 * a, j = jt + tx + 16 * b;
                        if (i < nb && j < nb) W[(size_t)i * ldw + j] = acc[a][b];
                    }
            }
            __syncthreads();
        }
    }
}

__global__ void __launch_bounds__(kBigThreads)
lu_big_f64(const int32_t *__restrict__ job_block, const int64_t *__restrict__ job_prefix, int njobs,
           int64_t nitems_range, const int2 *__restrict__ list, const int *__restrict__ list_count,
           const BlockDev *__restrict__ blocks, const InstDev *__restrict__ insts,
           const double2 *__restrict__ Hpool, const int32_t *__restrict__ rbpool,
           const double *__restrict__ eigpool, double2 *__restrict__ work, int ldw,
           double2 *__restrict__ contrib, int *__restrict__ status)
{
    extern __shared__ double2 s_dyn[];
    double2 *s_panel = s_dyn;                       // ldw x kPanel
    double2 *s_utile = s_panel + (size_t)ldw * kPanel;  // kPanel x 64
    double2 *s_piv = s_utile + kPanel * 64;          // ldw
    double2 *s_d = s_piv + ldw;                      // ldw
    __shared__ double2 s_w[kMaxBins];
    __shared__ double2 s_red[kBigThreads / 64 + 1];
    __shared__ int s_bad;

    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4;
    double2 *__restrict__ W = work + (size_t)blockIdx.x * ldw * ldw;
    const int64_t nitems = list ? (int64_t)*list_count : nitems_range;

    for (int64_t item = blockIdx.x; item < nitems; item += gridDim.x) {
        int bi;
        int64_t pt;
        if (list) {
            const int2 e = list[item];
            bi = e.x;
            pt = e.y;
        } else {
            const int job = find_job(job_prefix, njobs, item);
            bi = job_block[job];
            pt = item - job_prefix[job];
        }
        const BlockDev B = blocks[bi];
        const InstDev &I = insts[B.inst];
        const int nb = B.nb;
        __syncthreads();
        if (tid < I.L) point_w(I, pt, tid, s_w[tid]);
        if (tid == 0) s_bad = 0;
        __syncthreads();
        for (int i = tid; i < nb; i += kBigThreads) {
            const int b = rbpool[B.rb_off + i];
            s_d[i] = b < 0 ? cmk(1.0, 0.0) : s_w[b];
        }
        __syncthreads();
        const double2 *__restrict__ Hs = Hpool + B.h_off;
        if (B.hs_stride) Hs += (int64_t)point_k(I, pt, B.schur_axis) * B.hs_stride;
        for (int64_t e = tid; e < (int64_t)nb * nb; e += kBigThreads) {
            const int i = (int)(e / nb), j = (int)(e % nb);
            const double2 h = Hs[e];
            const double2 d = s_d[i];
            double2 v = cmk(i == j ? 1.0 : 0.0, 0.0);
            v.x -= d.x * h.x - d.y * h.y;
            v.y -= d.x * h.y + d.y * h.x;
            W[(size_t)i * ldw + j] = v;
        }
        __syncthreads();

        for (int k0 = 0; k0 < nb; k0 += kPanel) {
            const int kb = min(kPanel, nb - k0);
            const int mrows = nb - k0;
            // panel -> LDS
            for (int e = tid; e < mrows * kPanel; e += kBigThreads) {
                const int i = e / kPanel, t = e % kPanel;
                s_panel[e] = t < kb ? W[(size_t)(k0 + i) * ldw + k0 + t] : cmk(0.0, 0.0);
            }
            __syncthreads();
            for (int kk = 0; kk < kb; ++kk) {
                const double2 d = s_panel[kk * kPanel + kk];
                if (tid == 0) {
                    s_piv[k0 + kk] = d;
                    // pivots of S lie in the right half-plane; the border's (1 - 2E) need not
                    if (!isfinite(d.x) || !isfinite(d.y) || (k0 + kk < nb - B.bordered && !(d.x > 0.0))) s_bad = 1;
                }
                const double2 dinv = cinv(d);
                for (int i = kk + 1 + tid; i < mrows; i += kBigThreads) {
                    const double2 l = cmul(s_panel[i * kPanel + kk], dinv);
                    s_panel[i * kPanel + kk] = l;
                    for (int t = kk + 1; t < kb; ++t)
                        s_panel[i * kPanel + t] = cfnms(s_panel[i * kPanel + t], l, s_panel[kk * kPanel + t]);
                }
                __syncthreads();
            }
            const int j0 = k0 + kb;
            if (j0 >= nb) break;
            // U12 = L11^-1 A12 (unit lower triangular solve), in place in W
            for (int j = j0 + tid; j < nb; j += kBigThreads) {
                double2 x[kPanel];
                #pragma unroll
                for (int t = 0; t < kPanel; ++t) x[t] = t < kb ? W[(size_t)(k0 + t) * ldw + j] : cmk(0.0, 0.0);
                #pragma unroll
                for (int t = 1; t < kPanel; ++t) {
                    #pragma unroll
                    for (int s2 = 0; s2 < t; ++s2) x[t] = cfnms(x[t], s_panel[t * kPanel + s2], x[s2]);
                }
                #pragma unroll
                for (int t = 0; t < kPanel; ++t)
                    if (t < kb) W[(size_t)(k0 + t) * ldw + j] = x[t];
            }
            __syncthreads();
            // trailing update A22 -= L21 U12
            for (int jt = j0; jt < nb; jt += 64) {
                for (int e = tid; e < kPanel * 64; e += kBigThreads) {
                    const int t = e / 64, jj = jt + (e % 64);
                    s_utile[e] = (t < kb && jj < nb) ? W[(size_t)(k0 + t) * ldw + jj] : cmk(0.0, 0.0);
                }
                __syncthreads();
                for (int it = j0; it < nb; it += 64) {
                    double2 acc[4][4];
                    #pragma unroll
                    for (int a = 0; a < 4; ++a)
                        #pragma unroll
                        for (int b = 0; b < 4; ++b) {
                            const int i = it + ty + 16 * a, j = jt + tx + 16 * b;
                            acc[a][b] = (i < nb && j < nb) ? W[(size_t)i * ldw + j] : cmk(0.0, 0.0);
                        }
                    for (int t = 0; t < kb; ++t) {
                        double2 l[4], u[4];
                        #pragma unroll
                        for (int a = 0; a < 4; ++a) {
                            const int i = it + ty + 16 * a;
                            l[a] = i < nb ? s_panel[(i - k0) * kPanel + t] : cmk(0.0, 0.0);
                        }
                        #pragma unroll
                        for (int b = 0; b < 4; ++b) u[b] = s_utile[t * 64 + tx + 16 * b];
                        #pragma unroll
                        for (int a = 0; a < 4; ++a)
                            #pragma unroll
                            for (int b = 0; b < 4; ++b) acc[a][b] = cfnms(acc[a][b], l[a], u[b]);
                    }
                    #pragma unroll
                    for (int a = 0; a < 4; ++a)
                        #pragma unroll
                        for (int b = 0; b < 4; ++b) {
                            const int i = it + ty + 16 * a, j = jt + tx + 16 * b;
                            if (i < nb && j < nb) W[(size_t)i * ldw + j] = acc[a][b];
                        }
                }
                __syncthreads();
            }
        }
        __syncthreads();
        const int nlog = nb - B.bordered;
        double2 acc = cmk(0.0, 0.0);
        for (int i = tid; i < nlog; i += kBigThreads) {
            const double2 lg = clog(s_piv[i]);
            acc.x += lg.x;
            acc.y += lg.y;
        }
        if (B.n_eig > 0) {
            const double2 wa = s_w[B.schur_axis];
            const double *__restrict__ lam = eigpool + B.eig_off;
            for (int i = tid; i < B.n_eig; i += kBigThreads) {
                const double2 lg = clog(cmk(1.0 - wa.x * lam[i], -wa.y * lam[i]));
                acc.x += lg.x;
                acc.y += lg.y;
            }
        }
        acc = block_sum<kBigThreads>(acc, s_red);
        if (tid == 0) {
            double2 res = cmk(-0.5 * acc.x, -0.5 * acc.y);
            if (B.bordered) {
                const double2 p = s_piv[nb - 1];
                res.x += 0.5 * (1.0 - p.x);
                res.y += 0.5 * (0.0 - p.y);
            }
            contrib[I.c_off + pt * I.nblocks + B.blk] = res;
            if (s_bad) atomicOr(status, 1);
        }
    }
}

// ---------------------------------------------------------------------------
// Pair route (PairDev).  For every (k_A, k_P) pair, with C = C(w_A) and rows
// and columns in the order perm (bin P first),
//     F = E - D C,  E = diag(1 on bin-P rows, 0 on bin-B rows),
//                   D = diag(w_P on bin-P rows, -1 on bin-B rows),
// i.e. F = [[I - w_P C_PP, -w_P C_PB], [C_BP, C_BB]].  A partial unpivoted LU
// over the nP pivots of bin P (big_lu_steps) leaves S = C_BB + w_P C_BP
// (I - w_P C_PP)^-1 C_PB in the trailing block; S goes to the matrix pool for
// the Hessenberg reduction, and sum Log(pivots) + sum_i Log(1 - w_A lambda_i)
// goes to the pair's constant.  I - w_P C_PP is a principal block of the
// accretive I - D C(w_A), so its pivots lie in the right half-plane and the
// sum of their principal logarithms is the continuous branch.  One workgroup
// per pair, persistent; F lives in a per-workgroup global workspace.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBigThreads)
pair_schur_f64(const PairDev *__restrict__ jobs, const int64_t *__restrict__ prefix, int njobs, int64_t npairs,
               double2 *__restrict__ pool, const int32_t *__restrict__ permpool, const double *__restrict__ eigpool,
               double2 *__restrict__ work, int ldw, double2 *__restrict__ eigc, int *__restrict__ status)
{
    extern __shared__ double2 s_dyn[];
    double2 *s_panel = s_dyn;                           // ldw x kPanel
    double2 *s_utile = s_panel + (size_t)ldw * kPanel;  // kPanel x 64
    double2 *s_piv = s_utile + kPanel * 64;             // ldw
    int *s_perm = reinterpret_cast<int *>(s_piv + ldw); // ldw
    __shared__ double2 s_red[kBigThreads / 64 + 1];
    __shared__ int s_bad;

    const int tid = threadIdx.x;
    double2 *__restrict__ W = work + (size_t)blockIdx.x * ldw * ldw;
    for (int64_t p = blockIdx.x; p < npairs; p += gridDim.x) {
        const int job = find_job(prefix, njobs, p);
        const PairDev J = jobs[job];
        const int64_t lp = p - prefix[job];
        const int kA = (int)(lp / J.dP), kP = (int)(lp % J.dP);
        const int n = J.n, nP = J.nP, nH = J.n - J.nP;
        double sn, cs;
        { const double2 t_ = grid_w(kP, J.GP, J.rho); cs = t_.x; sn = t_.y; }
        const double2 wP = cmk(cs, sn);
        __syncthreads();  // the previous pair is done with s_perm, s_piv and W
        for (int i = tid; i < n; i += kBigThreads) s_perm[i] = permpool[J.perm_off + i];
        if (tid == 0) s_bad = 0;
        __syncthreads();
        const double2 *__restrict__ C = pool + J.c_off + (int64_t)kA * J.hs_stride;
        for (int64_t e = tid; e < (int64_t)n * n; e += kBigThreads) {
            const int i = (int)(e / n), j = (int)(e % n);
            const double2 h = C[(int64_t)s_perm[i] * n + s_perm[j]];
            double2 v = h;
            if (i < nP) {
                const double2 t = cmul(wP, h);
                v = cmk((i == j ? 1.0 : 0.0) - t.x, -t.y);
            }
            W[(size_t)i * ldw + j] = v;
        }
        __syncthreads();
        big_lu_steps(W, ldw, n, nP, nP, s_panel, s_utile, s_piv, &s_bad);
        __syncthreads();
        double2 *__restrict__ S = pool + J.s_off + lp * nH * nH;
        for (int64_t e = tid; e < (int64_t)nH * nH; e += kBigThreads) {
            const int i = (int)(e / nH), j = (int)(e % nH);
            S[e] = W[(size_t)(nP + i) * ldw + nP + j];
        }
        double2 acc = cmk(0.0, 0.0);
        for (int i = tid; i < nP; i += kBigThreads) {
            const double2 lg = clog(s_piv[i]);
            acc.x += lg.x;
            acc.y += lg.y;
        }
        { const double2 t_ = grid_w(kA, J.GA, J.rho); cs = t_.x; sn = t_.y; }
        const double *__restrict__ lam = eigpool + J.eig_off;
        for (int i = tid; i < J.n_eig; i += kBigThreads) {
            const double2 lg = clog(cmk(1.0 - cs * lam[i], -sn * lam[i]));
            acc.x += lg.x;
            acc.y += lg.y;
        }
        acc = block_sum<kBigThreads>(acc, s_red);
        if (tid == 0) {
            eigc[J.ec_off + lp] = acc;
            if (s_bad) atomicOr(status, 1);
        }
    }
}

// ---------------------------------------------------------------------------
// Schur matrices of the remaining bins after eliminating bin A through the
// eigenbasis of H_AA (Hermitian, H_AA = V diag(lambda) V^H):
//     C(w_A) = H_BB + P diag(f) Q,  f_i = w_A / (1 - w_A lambda_i),
// so that I - D_B C(w_A) is the Schur complement of S(w) on the other bins and
// det S = prod_i (1 - w_A lambda_i) det(I - D_B C(w_A)).
// One workgroup per (job, k, 4-row block of C): many small workgroups, since
// each thread walks the whole inner dimension.
// ---------------------------------------------------------------------------
constexpr int kSchurRows = 4;

__global__ void __launch_bounds__(256)
schur_build_f64(const SchurDev *__restrict__ jobs, const int64_t *__restrict__ job_prefix, int njobs,
                const double2 *__restrict__ pool_in, const double *__restrict__ eigpool,
                double2 *__restrict__ pool_out, float2 *__restrict__ pool32_out)
{
    extern __shared__ double2 s_dyn[];
    const int job = find_job(job_prefix, njobs, blockIdx.x);
    const SchurDev J = jobs[job];
    const int64_t local = blockIdx.x - job_prefix[job];
    const int nrb = (J.nB + kSchurRows - 1) / kSchurRows;
    const int k = (int)(local / nrb);
    const int r0 = (int)(local % nrb) * kSchurRows;
    double2 *s_f = s_dyn;                 // nA
    double2 *s_pf = s_f + J.nA;           // kSchurRows x nA
    const double2 w = grid_w(k, J.Gax, J.rho);
    const double *lam = eigpool + J.eig_off;
    for (int i = threadIdx.x; i < J.nA; i += blockDim.x)
        s_f[i] = cmul(w, cinv(cmk(1.0 - w.x * lam[i], -w.y * lam[i])));
    __syncthreads();
    const double2 *P = pool_in + J.p_off;
    for (int e = threadIdx.x; e < kSchurRows * J.nA; e += blockDim.x) {
        const int rr = e / J.nA, i = e % J.nA;
        const int r = r0 + rr;
        s_pf[e] = r < J.nB ? cmul(P[(int64_t)r * J.nA + i], s_f[i]) : cmk(0.0, 0.0);
    }
    __syncthreads();
    const double2 *Q = pool_in + J.q_off;
    const double2 *Hbb = pool_in + J.hbb_off;
    double2 *C = pool_out + J.c_off + (int64_t)k * J.nB * J.nB;
    for (int col = threadIdx.x; col < J.nB; col += blockDim.x) {
        double2 acc[kSchurRows];
        #pragma unroll
        for (int rr = 0; rr < kSchurRows; ++rr) {
            const int r = r0 + rr;
            acc[rr] = r < J.nB ? Hbb[(int64_t)r * J.nB + col] : cmk(0.0, 0.0);
        }
        // terms in the order of i; the loads of four rows of Q go out together
        auto terms = [&](int i, double2 q) {
            #pragma unroll
            for (int rr = 0; rr < kSchurRows; ++rr) {
                const double2 pf = s_pf[rr * J.nA + i];
                acc[rr].x = fma(pf.x, q.x, acc[rr].x);
                acc[rr].x = fma(-pf.y, q.y, acc[rr].x);
                acc[rr].y = fma(pf.x, q.y, acc[rr].y);
                acc[rr].y = fma(pf.y, q.x, acc[rr].y);
            }
        };
        int i = 0;
        for (; i + 4 <= J.nA; i += 4) {
            double2 q[4];
            #pragma unroll
            for (int u = 0; u < 4; ++u) q[u] = Q[(int64_t)(i + u) * J.nB + col];
            #pragma unroll
            for (int u = 0; u < 4; ++u) terms(i + u, q[u]);
        }
        for (; i < J.nA; ++i) terms(i, Q[(int64_t)i * J.nB + col]);
        #pragma unroll
        for (int rr = 0; rr < kSchurRows; ++rr) {
            const int r = r0 + rr;
            if (r < J.nB) {
                const int64_t o = (int64_t)r * J.nB + col;
                C[o] = acc[rr];
                if (pool32_out) {
                    float2 f;
                    f.x = (float)acc[rr].x;
                    f.y = (float)acc[rr].y;
                    pool32_out[J.c_off + (int64_t)k * J.nB * J.nB + o] = f;
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Kernel H: blocks whose rows left after the eigenbasis elimination of bin A
// all belong to one bin B.  Then D_B = w_B I, and for every value of w_A,
//     det(I - w_B C(w_A)) = det(I - w_B Hh),   Hh = Q^H C(w_A) Q upper Hessenberg,
// with Q a product of Householder reflections.  hess_reduce_f64 brings each
// C(w_A) to that form (in place); hess_det_f64 factorises I - w_B Hh for
// every w_B by unpivoted LU of a Hessenberg matrix (O(n^2)); hess_scatter
// copies the per-(w_A, w_B) values to the evaluated points.  I - w_B C(w_A)
// is the Schur complement of S after eliminating A, so it is accretive, and
// so is any unitary similarity of it: every pivot has Re > 0 and the sum of
// the principal logarithms of the pivots is the continuous branch.
// ---------------------------------------------------------------------------
constexpr int kHessDetThreads = 256;  // 4 waves x 4 points, 16 lanes per point

// TY x TX thread grid (TY = 16 or 32), ty = tid % TY and tx = tid / TY:
// element (i, j) in thread (i mod TY, j mod TX), register (i / TY, j / TX).
// Matrix column j is held by TY consecutive lanes of one wave (one DPP row,
// or two), so sums down a column run in DPP.  RMAX = TY R rows and CMAX =
// TX SC columns are held, orders n <= min(RMAX, CMAX).  The y partials (one
// per column thread) number TX per row and the w partials (one per DPP quad)
// TY / 4 per column.
template <int TY, int TX, int R, int SC>
struct HessLds {
    static constexpr int NT = TX * TY;
    static constexpr int RMAX = TY * R;
    static constexpr int CMAX = TX * SC;
    static constexpr int NMAX = RMAX < CMAX ? RMAX : CMAX;
    static constexpr int XMAX = RMAX > CMAX ? RMAX : CMAX;
    static constexpr int PYS = RMAX + 1;  // padded strides of the partial sums
    static constexpr int PWS = CMAX + 1;
    double2 x[2][XMAX];                    // v of step k (zero outside rows k+1..n-1), by step parity
    double beta[2];                        // 2 / |v|^2 of step k, by step parity
    double2 PW[TY / 4][PWS];               // partials of w_j = sum_i conj(v_i) a_ij, per 4 thread rows
    double2 PY[32][PYS];                   // partials of y_i = sum_j a_ij v_j, per thread column (TX <= 32
                                           // rows used; 32 so that it can stage the matrix)
    double2 PS[NT];                        // partials of s = v^H A v, per thread
    double2 W[CMAX], Y[RMAX];
    double2 S;
    double2 red[NT / 64 + 1];
};

// x from lane (lane ^ 1) (CTRL 0xB1) or (lane ^ 2) (CTRL 0x4E) of the same
// quad (DPP quad_perm), or from the mirrored lane of the same half row
// (0x141, lane 7 - i of each 8) or row (0x140, lane 15 - i of each 16)
template <int CTRL>
__device__ __forceinline__ double quad_swap(double x) {
    const int2 u = __builtin_bit_cast(int2, x);
    int2 v;
    v.x = __builtin_amdgcn_mov_dpp(u.x, CTRL, 0xf, 0xf, true);
    v.y = __builtin_amdgcn_mov_dpp(u.y, CTRL, 0xf, 0xf, true);
    return __builtin_bit_cast(double, v);
}

// Sum over the 16 lanes of each DPP row; every lane of the row gets the same
// value (each level adds two equal-order partial sums, and a + b = b + a).
__device__ __forceinline__ double row16_sum(double x) {
    x += quad_swap<0xB1>(x);
    x += quad_swap<0x4E>(x);
    x += quad_swap<0x141>(x);
    x += quad_swap<0x140>(x);
    return x;
}

// Sum over the TY lanes that hold one matrix column: one DPP row (TY = 16),
// or two adjacent rows (TY = 32), whose row sums a 16-lane swap adds.
template <int TY>
__device__ __forceinline__ double col_sum(double x) {
    x = row16_sum(x);
    if constexpr (TY == 32) {
        const int2 u = __builtin_bit_cast(int2, x);
        const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)u.x, (unsigned)u.x, false, false);
        const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)u.y, (unsigned)u.y, false, false);
        const double a = __builtin_bit_cast(double, make_uint2(lo[0], hi[0]));
        const double b = __builtin_bit_cast(double, make_uint2(lo[1], hi[1]));
        x = a + b;
    }
    return x;
}

// x of lane LANE of the wave (wave-uniform result)
template <int LANE>
__device__ __forceinline__ double lane_read(double x) {
    const int2 u = __builtin_bit_cast(int2, x);
    int2 v;
    v.x = __builtin_amdgcn_readlane(u.x, LANE);
    v.y = __builtin_amdgcn_readlane(u.y, LANE);
    return __builtin_bit_cast(double, v);
}

// Reflector of step k, computed by the lanes that hold column k (register
// column S): x = column k below the diagonal goes to L.x[par] (zero at rows
// <= k and >= n), then v_1 = x_1 - alpha with alpha = -(x_1/|x_1|) |x|
// replaces x_1 there, and beta = 2 / |v|^2 = 1 / (|x| (|x| + |x_1|)) goes to
// L.beta[par].  All TY lanes of the column must be active.
template <int TY, int TX, int R, int SC, int S>
__device__ __forceinline__ void hess_reflector(HessLds<TY, TX, R, SC> &L, const double2 (&a)[R][SC], int k, int n,
                                               int par, int ty) {
    double acc = 0.0;
    double2 x1 = cmk(0.0, 0.0);
    double2 *xr = &L.x[par][ty];
    #pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = ty + TY * r;
        const bool in = i > k && i < n;
        const double2 xi = cmk(in ? a[r][S].x : 0.0, in ? a[r][S].y : 0.0);
        xr[TY * r] = xi;
        acc = fma(xi.x, xi.x, fma(xi.y, xi.y, acc));
        x1.x = i == k + 1 ? xi.x : x1.x;
        x1.y = i == k + 1 ? xi.y : x1.y;
    }
    const double xn = sqrt(col_sum<TY>(acc));
    x1.x = col_sum<TY>(x1.x);  // one nonzero term
    x1.y = col_sum<TY>(x1.y);
    const double ax1 = sqrt(x1.x * x1.x + x1.y * x1.y);
    if (ty == ((k + 1) & (TY - 1))) {
        const double2 ph = ax1 > 0.0 ? cmk(x1.x / ax1, x1.y / ax1) : cmk(1.0, 0.0);
        L.x[par][k + 1] = cmk(ph.x * (ax1 + xn), ph.y * (ax1 + xn));
        L.beta[par] = xn > 0.0 ? 1.0 / (xn * (xn + ax1)) : 0.0;
    }
}

// One Householder step k (column k) of hess_reduce_f64, R0 = k / TY and
// S0 = k / TX.  Register rows r < R0 hold only rows < k, where v vanishes;
// register columns s < S0 hold only columns < k, where v vanishes, so their
// entries on or above the subdiagonal (rows i <= j + 1 <= k) do not change.  The
// terms they would carry are left out at compile time.  Column k becomes
// (alpha, O(eps |x|), ...) below the diagonal; what is left below the
// subdiagonal never reaches the Hessenberg part (v vanishes on those rows and
// columns in every later step) and is written out as zero.
template <int TY, int TX, int R, int SC, int R0, int S0>
__device__ __forceinline__ void hess_step(HessLds<TY, TX, R, SC> &L, double2 (&a)[R][SC], int k, int n, int tid) {
    constexpr int NT = TX * TY, RMAX = TY * R, CMAX = TX * SC;
    const int par = k & 1, ty = tid & (TY - 1), tx = tid / TY;

    // A. reflector, by the lanes that hold column k
    if (tx == k % TX) hess_reflector<TY, TX, R, SC, S0>(L, a, k, n, par, ty);
    __syncthreads();
    const double beta = L.beta[par];

    // per-thread LDS bases; register rows and columns are constant offsets
    const double2 *xr = &L.x[par][ty], *xc = &L.x[par][tx];
    double2 *pyr = &L.PY[tx][ty], *pwr = &L.PW[ty / 4][tx];
    const double2 *yr = &L.Y[ty], *wc = &L.W[tx];

    // B. partial sums of y = A v (all rows), w = v^H A and s = v^H y
    double2 ps = cmk(0.0, 0.0);
    {
        double2 vj[SC];
        #pragma unroll
        for (int s = S0; s < SC; ++s) vj[s] = xc[TX * s];
        #pragma unroll
        for (int r = 0; r < R; ++r) {
            double2 py = cmk(0.0, 0.0);
            #pragma unroll
            for (int s = S0; s < SC; ++s) py = cfma(a[r][s], vj[s], py);
            pyr[TY * r] = py;
            if (r >= R0) ps = cfma_conj(xr[TY * r], py, ps);
        }
    }
    {
        double2 pw[SC];
        #pragma unroll
        for (int s = S0; s < SC; ++s) pw[s] = cmk(0.0, 0.0);
        #pragma unroll
        for (int r = R0; r < R; ++r) {
            const double2 vi = xr[TY * r];
            #pragma unroll
            for (int s = S0; s < SC; ++s) pw[s] = cfma_conj(vi, a[r][s], pw[s]);
        }
        // sums over each DPP quad (four thread rows of one column); the four
        // lanes store the same value to the same place, which keeps the code
        // free of branches
        #pragma unroll
        for (int s = S0; s < SC; ++s) {
            pw[s].x += quad_swap<0xB1>(pw[s].x);
            pw[s].y += quad_swap<0xB1>(pw[s].y);
            pw[s].x += quad_swap<0x4E>(pw[s].x);
            pw[s].y += quad_swap<0x4E>(pw[s].y);
        }
        #pragma unroll
        for (int s = S0; s < SC; ++s) pwr[TX * s] = pw[s];
    }
    L.PS[tid] = ps;
    __syncthreads();

    // C. reductions, each in a fixed order: y_i by lane i (TX partials, four
    // loads at a time), w_j by lane RMAX + j (TY / 4 partials), s by the last
    // wave
    {
        if (tid < RMAX) {
            constexpr int PYS = HessLds<TY, TX, R, SC>::PYS;
            const double2 *row = &L.PY[0][tid];
            double2 t = cmk(0.0, 0.0);
            #pragma unroll
            for (int q = 0; q < TX; q += 4) {
                const double2 u0 = row[q * PYS], u1 = row[(q + 1) * PYS];
                const double2 u2 = row[(q + 2) * PYS], u3 = row[(q + 3) * PYS];
                t.x += (u0.x + u1.x) + (u2.x + u3.x);
                t.y += (u0.y + u1.y) + (u2.y + u3.y);
            }
            L.Y[tid] = t;
        }
        const int jw = tid - RMAX;
        if (jw >= TX * S0 && jw < CMAX) {
            constexpr int PWS = HessLds<TY, TX, R, SC>::PWS;
            const double2 *col = &L.PW[0][jw];
            double2 t = cmk(0.0, 0.0);
            #pragma unroll
            for (int q = 0; q < TY / 4; q += 4) {
                const double2 u0 = col[q * PWS], u1 = col[(q + 1) * PWS];
                const double2 u2 = col[(q + 2) * PWS], u3 = col[(q + 3) * PWS];
                t.x += (u0.x + u1.x) + (u2.x + u3.x);
                t.y += (u0.y + u1.y) + (u2.y + u3.y);
            }
            L.W[jw] = t;
        }
    }
    if (tid >= NT - 64) {
        const int lane = tid & 63;
        double2 t0 = cmk(0.0, 0.0), t1 = cmk(0.0, 0.0);
        #pragma unroll
        for (int q = 0; q < NT / 64; q += 2) {
            t0.x += L.PS[lane + 64 * q].x;
            t0.y += L.PS[lane + 64 * q].y;
            t1.x += L.PS[lane + 64 * (q + 1)].x;
            t1.y += L.PS[lane + 64 * (q + 1)].y;
        }
        // DPP row sums, then the four rows in a fixed order
        const double tx0 = row16_sum(t0.x + t1.x), ty0 = row16_sum(t0.y + t1.y);
        const double sx = (lane_read<0>(tx0) + lane_read<16>(tx0)) + (lane_read<32>(tx0) + lane_read<48>(tx0));
        const double sy = (lane_read<0>(ty0) + lane_read<16>(ty0)) + (lane_read<32>(ty0) + lane_read<48>(ty0));
        if (lane == 0) L.S = cmk(sx, sy);
    }
    __syncthreads();

    // D. A <- A - beta z v^H - beta v w with z = y - beta s v, one rank-1
    // term per pass
    const double2 sv = L.S;
    const double2 bs = cmk(beta * sv.x, beta * sv.y);
    {
        double2 cvj[SC];
        #pragma unroll
        for (int s = S0; s < SC; ++s) {
            const double2 v = xc[TX * s];
            cvj[s] = cmk(v.x, -v.y);
        }
        #pragma unroll
        for (int r = 0; r < R; ++r) {
            const double2 yi = yr[TY * r];
            double2 zi;  // beta z_i
            if (r >= R0) {
                const double2 bsv = cmul(bs, xr[TY * r]);
                zi = cmk(beta * (yi.x - bsv.x), beta * (yi.y - bsv.y));
            } else {
                zi = cmk(beta * yi.x, beta * yi.y);
            }
            #pragma unroll
            for (int s = S0; s < SC; ++s) a[r][s] = cfnms(a[r][s], zi, cvj[s]);
        }
    }
    {
        double2 wj[SC];
        #pragma unroll
        for (int s = S0; s < SC; ++s) wj[s] = wc[TX * s];
        #pragma unroll
        for (int r = R0; r < R; ++r) {
            const double2 vi = xr[TY * r];
            const double2 bvi = cmk(beta * vi.x, beta * vi.y);
            #pragma unroll
            for (int s = S0; s < SC; ++s) a[r][s] = cfnms(a[r][s], bvi, wj[s]);
        }
    }
}

// Steps k with (k / TY, k / TX) = (R0, S0), then the following values: one
// loop per pair, so that each loop body is straight-line code.
template <int TY, int TX, int R, int SC, int R0, int S0>
__device__ __forceinline__ void hess_steps_from(HessLds<TY, TX, R, SC> &L, double2 (&a)[R][SC], int n, int tid) {
    constexpr int RE = TY * (R0 + 1), SE = TX * (S0 + 1);  // where R0, S0 change
    const int k_lo = max(TY * R0, TX * S0), k_hi = min(min(RE, SE), n - 2);
    for (int k = k_lo; k < k_hi; ++k) hess_step<TY, TX, R, SC, R0, S0>(L, a, k, n, tid);
    constexpr int R1 = R0 + (RE <= SE ? 1 : 0), S1 = S0 + (SE <= RE ? 1 : 0);
    if constexpr (R1 < R && S1 < SC) hess_steps_from<TY, TX, R, SC, R1, S1>(L, a, n, tid);
}

// Householder reduction to upper Hessenberg form of C(w_A), one workgroup per
// (block, k_A).  Step k reflects column k: with v the Householder vector,
// beta = 2 / |v|^2, w = v^H A, y = A v and s = w v, the two-sided
// reflection is the rank-2 update A <- A - beta v w - beta (y - beta s v) v^H,
// so both sums come from one pass over A.  Every element a thread holds goes
// through the same straight-line code (v is zero outside rows k+1..n-1, in
// LDS, padding included); only whole register rows and columns that carry no
// terms are left out (hess_step).  Entries below the subdiagonal are written
// as zero.  Also writes sum_i Log(1 - w_A lambda_i) of the eliminated bin.
template <int TY, int TX, int R, int SC>
__global__ void __launch_bounds__(TX * TY) hess_reduce_f64(const HessDev *__restrict__ jobs,
                                                                 const int64_t *__restrict__ prefix, int njobs,
                                                                 double2 *__restrict__ pool,
                                                                 const double *__restrict__ eigpool,
                                                                 double2 *__restrict__ eigc)
{
    using Lds = HessLds<TY, TX, R, SC>;
    constexpr int NMAX = Lds::NMAX, RMAX = Lds::RMAX, CMAX = Lds::CMAX, XMAX = Lds::XMAX;
    constexpr int NT = Lds::NT;
    static_assert(NT >= 512, "reductions assume 512 threads or more");
    static_assert(RMAX + CMAX <= NT - 64 && TX % 4 == 0 && TX <= 32, "reduction threads overlap");
    static_assert(TY == 16 || TY == 32, "one matrix column per one or two 16-lane DPP rows");
    extern __shared__ __align__(16) unsigned char hess_raw[];
    Lds &L = *reinterpret_cast<Lds *>(hess_raw);
    const int job = find_job(prefix, njobs, blockIdx.x);
    const HessDev J = jobs[job];
    const int kA = (int)(blockIdx.x - prefix[job]);
    const int n = J.n;
    const int tid = threadIdx.x, ty = tid & (TY - 1), tx = tid / TY;
    double2 *__restrict__ C = pool + J.c_off + (int64_t)kA * n * n;

    // v is read at every index < XMAX; indices >= RMAX are never written
    for (int e = tid; e < 2 * XMAX; e += NT) (&L.x[0][0])[e] = cmk(0.0, 0.0);

    // The matrix moves between HBM and registers through LDS (the row-sum
    // partial buffer), CR register rows (CR TY matrix rows, contiguous in C)
    // at a time: plain coalesced copies, and few live addresses.
    constexpr int CR = (32 * Lds::PYS) / (NMAX * TY);
    static_assert(CR >= 1, "staging buffer too small");
    double2 *stage = &L.PY[0][0];
    double2 a[R][SC];
    #pragma unroll
    for (int c0 = 0; c0 < R; c0 += CR) {
        const int i0 = c0 * TY;
        const int rows = max(0, min(CR * TY, n - i0));
        for (int e = tid; e < rows * n; e += NT) stage[e] = C[(int64_t)i0 * n + e];
        __syncthreads();
        #pragma unroll
        for (int r = c0; r < c0 + CR && r < R; ++r)
            #pragma unroll
            for (int s = 0; s < SC; ++s) {
                const int i = ty + TY * r, j = tx + TX * s;
                const bool in = i < n && j < n;
                const double2 h = stage[in ? (i - i0) * n + j : 0];
                a[r][s] = in ? h : cmk(0.0, 0.0);
            }
        __syncthreads();
    }

    hess_steps_from<TY, TX, R, SC, 0, 0>(L, a, n, tid);

    __syncthreads();
    #pragma unroll
    for (int c0 = 0; c0 < R; c0 += CR) {
        const int i0 = c0 * TY;
        const int rows = max(0, min(CR * TY, n - i0));
        #pragma unroll
        for (int r = c0; r < c0 + CR && r < R; ++r)
            #pragma unroll
            for (int s = 0; s < SC; ++s) {
                const int i = ty + TY * r, j = tx + TX * s;
                if (i < n && j < n) stage[(i - i0) * n + j] = i > j + 1 ? cmk(0.0, 0.0) : a[r][s];
            }
        __syncthreads();
        for (int e = tid; e < rows * n; e += NT) C[(int64_t)i0 * n + e] = stage[e];
        __syncthreads();
    }

    // sum_i Log(1 - w_A lambda_i); a pair job's constant comes with its
    // Schur complement (pair_schur_f64)
    if (J.axP >= 0) return;
    double sn, cs;
    { const double2 t_ = grid_w(kA, J.GA, J.rho); cs = t_.x; sn = t_.y; }
    const double *__restrict__ lam = eigpool + J.eig_off;
    double2 acc = cmk(0.0, 0.0);
    for (int i = tid; i < J.n_eig; i += NT) {
        const double2 lg = clog(cmk(1.0 - cs * lam[i], -sn * lam[i]));
        acc.x += lg.x;
        acc.y += lg.y;
    }
    acc = block_sum<NT>(acc, L.red);
    if (tid == 0) eigc[J.ec_off + kA] = acc;
}

template <int K>
__device__ __forceinline__ double dpp_bcast64(double x) {  // lane K of each 16-lane row
    const int2 u = __builtin_bit_cast(int2, x);
    int2 v;
    v.x = __builtin_amdgcn_mov_dpp(u.x, 0x150 + K, 0xf, 0xf, true);
    v.y = __builtin_amdgcn_mov_dpp(u.y, 0x150 + K, 0xf, 0xf, true);
    return __builtin_bit_cast(double, v);
}

// Argument of x + iy to within 0.004 rad: atan(t) ~ t (pi/4 + 0.273 (1 - t))
// on [0, 1], folded into the other octants.
__device__ __forceinline__ float rough_arg(float x, float y) {
    const float ax = fabsf(x), ay = fabsf(y);
    const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
    const float t = mx > 0.0f ? mn * __builtin_amdgcn_rcpf(mx) : 0.0f;
    float r = t * fmaf(0.273f, 1.0f - t, 0.78539816f);
    if (ay > ax) r = 1.57079633f - r;
    if (x < 0.0f) r = 3.14159265f - r;
    return y < 0.0f ? -r : r;
}

// Per-point state of the Hessenberg factorisation (see hess_det_f64).
template <int MB>
struct HessDetState {
    const double2 *__restrict__ Hh;
    const double2 *blk;         // LDS: rows 16 M + 1 .. 16 M + 16, columns 16 M .. (stride 16 MB)
    int n, e;                   // order, lane within the point's 16 lanes
    double2 w;                  // w_B
    double2 u[MB];              // row k of U: u_j in slot j / 16 of lane j % 16
    double argsum, logsum;      // sum of Log(pivot) over the closed groups
    double2 prod;               // product of the pivots of the open group
    float aest;                 // rough sum of their arguments
    int ngrp;                   // pivots in the open group
    bool bad;                   // a pivot left the right half-plane (or was NaN)

    __device__ __forceinline__ double2 hload(int row, int j) const {
        const bool in = row < n && j < n;
        const double2 h = Hh[in ? (int64_t)row * n + j : 0];
        return in ? h : cmk(0.0, 0.0);
    }
    // Hh[16 M + E0 + 1][e + 16 q] from the staged block of block M (zero
    // outside the matrix)
    template <int M, int E0>
    __device__ __forceinline__ double2 hblk(int q) const {
        return blk[E0 * 16 * MB + e + 16 * (q - M)];
    }
    __device__ __forceinline__ double2 mrow(int row, int j, double2 h) const {  // (I - w Hh)[row][j]
        const double2 t = cmul(w, h);
        return cmk((row == j ? 1.0 : 0.0) - t.x, -t.y);
    }
    // Pivots are taken in groups of 16: the sum of their principal
    // arguments is the argument of their product up to a multiple of 2 pi,
    // which a rough running sum of the arguments (error < 0.004 rad each)
    // fixes.  One exact atan2 and one log per group.
    __device__ __forceinline__ void flush() {
        const double th = atan2(prod.y, prod.x);
        const double turns = rint(((double)aest - th) * 0.15915494309189535);  // 1 / (2 pi)
        argsum += fma(turns, 6.283185307179586, th);
        logsum += 0.5 * log(prod.x * prod.x + prod.y * prod.y);
        prod = cmk(1.0, 0.0);
        aest = 0.0f;
        ngrp = 0;
    }
    __device__ __forceinline__ void take(double2 p) {
        bad |= !(p.x > 0.0);
        prod = cmul(prod, p);
        aest += rough_arg((float)p.x, (float)p.y);
        if (++ngrp == 16) flush();
    }
    // step k = 16 M + E0: pivot u_k, multiplier M[k+1][k] / u_k, row k+1 of U
    // (slots q < M hold columns < k and are no longer needed)
    template <int M, int E0>
    __device__ __forceinline__ void step() {
        const int k = 16 * M + E0;
        if (k >= n - 1) return;
        const double2 piv = cmk(dpp_bcast64<E0>(u[M].x), dpp_bcast64<E0>(u[M].y));
        const double2 hm = hblk<M, E0>(M);
        const double2 hsub = cmk(dpp_bcast64<E0>(hm.x), dpp_bcast64<E0>(hm.y));  // Hh[k+1][k]
        const double2 t = cmul(w, hsub);
        const double2 l = cmul(cmk(-t.x, -t.y), cinv(piv));
        u[M] = cfnms(mrow(k + 1, e + 16 * M, hm), l, u[M]);
        #pragma unroll
        for (int q = M + 1; q < MB; ++q) {
            if (16 * q >= n) break;
            const int j = e + 16 * q;
            u[q] = cfnms(mrow(k + 1, j, hblk<M, E0>(q)), l, u[q]);
        }
        take(piv);
    }
    template <int M, int... E>
    __device__ __forceinline__ void block(std::integer_sequence<int, E...>) {
        (step<M, E>(), ...);
    }
};

// Staging of block M (rows 16 M + 1 .. 16 M + 16, columns 16 M ..) for the
// Hessenberg factorisation: thread (E, c0) loads row 16 M + 1 + E, columns
// 16 M + c0 + 16 i, zero outside the matrix; then writes them to LDS buffer
// M mod 2 (stride 16 MB).
template <int MB, int M>
__device__ __forceinline__ void hess_det_fetch(const double2 *__restrict__ Hh, int n, int E, int c0,
                                               double2 (&pf)[MB]) {
    const int row = 16 * M + 1 + E;
    #pragma unroll
    for (int i = 0; i < MB - M; ++i) {
        const int col = 16 * M + c0 + 16 * i;
        const bool in = row < n && col < n;
        const double2 h = Hh[in ? (int64_t)row * n + col : 0];
        pf[i] = in ? h : cmk(0.0, 0.0);
    }
}
template <int MB, int M>
__device__ __forceinline__ void hess_det_stage(double2 *lds, int E, int c0, const double2 (&pf)[MB]) {
    #pragma unroll
    for (int i = 0; i < MB - M; ++i) lds[((M & 1) * 16 + E) * 16 * MB + c0 + 16 * i] = pf[i];
}

// Blocks M, M + 1, .. of 16 pivot steps (nblk in all): the next block is
// fetched into registers while this one runs and staged after it.
template <int MB, int M>
__device__ __forceinline__ void hess_det_blocks(HessDetState<MB> &S, double2 *lds, double2 (&pf)[MB], int nblk,
                                                int E, int c0) {
    if (M >= nblk) return;
    if constexpr (M + 1 < MB) {
        if (M + 1 < nblk) hess_det_fetch<MB, M + 1>(S.Hh, S.n, E, c0, pf);
    }
    S.blk = lds + (M & 1) * 16 * 16 * MB;
    S.template block<M>(std::make_integer_sequence<int, 16>{});
    if constexpr (M + 1 < MB) {
        if (M + 1 < nblk) hess_det_stage<MB, M + 1>(lds, E, c0, pf);
    }
    __syncthreads();
    if constexpr (M + 1 < MB) hess_det_blocks<MB, M + 1>(S, lds, pf, nblk, E, c0);
}

// Per point: unpivoted LU of the upper Hessenberg matrix M = I - w_B Hh.
// Row k+1 of U is M[k+1, :] - (M[k+1][k] / u_k) u with u = row k of U, so
// only one row of U is live.  16 lanes per point (4 points per wave), lane e
// holding u_j for j = e + 16 m; block M of 16 steps is code of its own
// (hess_det_blocks), so that every register index is static.  The 16 points of a
// workgroup share one C(w_A): the 16 rows a block of steps reads are staged
// in LDS (two buffers; the next block is loaded into registers while the
// current one runs).  The principal logarithms of the pivots are summed per
// group of 16 (HessDetState::flush).  Writes
// -1/2 (sum Log pivots + sum_i Log(1 - w_A lambda_i)) per (k_A, k_B).
template <int MB>
__global__ void __launch_bounds__(kHessDetThreads) hess_det_f64(const HessDev *__restrict__ jobs,
                                                                const int64_t *__restrict__ prefix, int njobs,
                                                                const double2 *__restrict__ pool,
                                                                const double2 *__restrict__ eigc,
                                                                double2 *__restrict__ table,
                                                                int *__restrict__ status)
{
    static_assert(kHessDetThreads == 256, "staging maps 16 rows x 16 lanes");
    extern __shared__ __align__(16) double2 hd_lds[];  // [2][16][16 MB]
    const int job = find_job(prefix, njobs, blockIdx.x);
    const HessDev J = jobs[job];
    const int64_t local = blockIdx.x - prefix[job];
    const int nch = (J.dB + 15) >> 4;
    const int kA = (int)(local / nch), chunk = (int)(local % nch);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4;
    const int kB = chunk * 16 + wave * 4 + g;
    const bool valid = kB < J.dB;
    const int n = J.n;

    HessDetState<MB> S;
    S.Hh = pool + J.c_off + (int64_t)kA * n * n;
    S.n = n;
    S.e = lane & 15;
    double sn, cs;
    { const double2 t_ = grid_w(valid ? kB : 0, J.GB, J.rho); cs = t_.x; sn = t_.y; }
    S.w = cmk(cs, sn);
    #pragma unroll
    for (int q = 0; q < MB; ++q) {
        const int j = S.e + 16 * q;
        S.u[q] = j < n ? S.mrow(0, j, S.hload(0, j)) : cmk(0.0, 0.0);
    }
    S.argsum = S.logsum = 0.0;
    S.prod = cmk(1.0, 0.0);
    S.aest = 0.0f;
    S.ngrp = 0;
    S.bad = false;

    // block M of 16 steps: rows 16 M + 1 + E of the staged block come from
    // thread (E, c0) = (tid / 16, tid % 16), columns 16 M + c0 + 16 i
    const int nblk = (n - 1 + 15) >> 4;  // blocks of steps k = 0 .. n - 2
    double2 pf[MB];
    hess_det_fetch<MB, 0>(S.Hh, n, tid >> 4, tid & 15, pf);
    hess_det_stage<MB, 0>(hd_lds, tid >> 4, tid & 15, pf);
    __syncthreads();
    hess_det_blocks<MB, 0>(S, hd_lds, pf, nblk, tid >> 4, tid & 15);
    // last pivot u_{n-1}: slot (n - 1) / 16, lane (n - 1) % 16
    const int ml = (n - 1) >> 4, el = (n - 1) & 15;
    double2 last = S.u[0];
    #pragma unroll
    for (int q = 1; q < MB; ++q)
        if (q == ml) last = S.u[q];
    last.x = __shfl(last.x, g * 16 + el, 64);
    last.y = __shfl(last.y, g * 16 + el, 64);
    S.take(last);
    if (S.ngrp > 0) S.flush();
    if (valid && S.e == 0) {
        const double2 ec = eigc[J.ec_off + kA];
        table[J.t_off + (int64_t)kA * J.dB + kB] = cmk(-0.5 * (S.logsum + ec.x), -0.5 * (S.argsum + ec.y));
        // pivots of I - w_B Hh lie in the right half-plane (accretive, unitarily
        // similar to a Schur complement of S); an infinite one leaves a
        // non-finite sum
        if (S.bad || !isfinite(S.logsum) || !isfinite(S.argsum)) atomicOr(status, 1);
    }
}

// contrib of a Hessenberg block at every evaluated point of its instance
__global__ void __launch_bounds__(256) hess_scatter(const HessDev *__restrict__ jobs,
                                                    const int64_t *__restrict__ prefix, int njobs, int64_t total,
                                                    const InstDev *__restrict__ insts,
                                                    const double2 *__restrict__ table, double2 *__restrict__ contrib)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int job = find_job(prefix, njobs, t);
    const HessDev J = jobs[job];
    const InstDev &I = insts[J.inst];
    const int64_t pt = t - prefix[job];
    int kA = point_k(I, pt, J.axA);
    if (J.axP >= 0) kA = kA * J.dP + point_k(I, pt, J.axP);
    const int kB = point_k(I, pt, J.axB);
    contrib[I.c_off + pt * I.nblocks + J.blk] = table[J.t_off + (int64_t)kA * J.dB + kB];
}

// ---------------------------------------------------------------------------
// log G(w) = log Pr(0) + (constant) + sum over internal blocks of each
// block's contribution, then G = exp(log G).  One thread per evaluated point.
// ---------------------------------------------------------------------------
__global__ void combine_points(const InstDev *__restrict__ insts, const int64_t *__restrict__ inst_pt_prefix,
                               int n_inst, int64_t npts_total, const double2 *__restrict__ contrib,
                               double2 *__restrict__ logg, double2 *__restrict__ gval)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npts_total) return;
    const int i = find_job(inst_pt_prefix, n_inst, p);
    const InstDev &I = insts[i];
    if (I.nvar) return;  // density mode: density_expand writes log G and the point's values
    const int64_t lp = p - I.pt_off;
    double2 acc = cmk(I.logpr0_re, I.logpr0_im);
    const double2 *c = contrib + I.c_off + lp * I.nblocks;
    for (int b = 0; b < I.nblocks; ++b) {
        acc.x += c[b].x;
        acc.y += c[b].y;
    }
    logg[p] = acc;
    if (I.dft_log) {  // cumulants: the DFT takes log G itself
        gval[I.gv_off + lp] = acc;
        return;
    }
    double s, co;
    sincos(acc.y, &s, &co);
    const double m = exp(acc.x);
    gval[I.gv_off + lp] = cmk(m * co, m * s);
}

// ---------------------------------------------------------------------------
// One axis of the separable inverse DFT, for every instance that still has
// this axis:  out[o][b][i] = sum_k in[o][k][i] exp(-2 pi i k b / G).
// The last stage (axis 0, the half-grid axis) folds in the conjugate half:
// P(b) = (1/prod G) sum_{k_1 <= G_1/2} c_k Re(...) with c_k = 1 for k_1 = 0
// (and k_1 = G_1/2 when G_1 is even), 2 otherwise.
// ---------------------------------------------------------------------------

__global__ void dft_stage(const DftStageDev *__restrict__ st, const int64_t *__restrict__ prefix, int n,
                          int64_t total, const double2 *__restrict__ twpool, const double2 *__restrict__ in,
                          double2 *__restrict__ out, double *__restrict__ probs, double *__restrict__ err,
                          const int *__restrict__ status)
{
    // four lanes (one DPP quad) per output, lane c taking the terms k = c mod 4
    const int64_t q = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 2;
    const int c = (int)(threadIdx.x & 3);
    if (q >= total) return;  // whole quads leave together
    const int e = find_job(prefix, n, q);
    const DftStageDev S = st[e];
    const int64_t lq = q - prefix[e];
    const int64_t i = lq % S.inner;
    const int b = (int)((lq / S.inner) % S.Bout);
    const int64_t o = lq / (S.inner * S.Bout);
    const double2 *src = in + S.in_off + o * S.K * S.inner + i;
    const double2 *tw = twpool + S.tw_off;
    double2 acc = cmk(0.0, 0.0);
    auto term = [&](int k, double2 v, double2 t) {
        if (S.final_stage && !S.density) {
            const double wk = (k == 0 || 2 * k == S.G) ? 1.0 : 2.0;
            v.x *= wk;
            v.y *= wk;
        }
        acc.x = fma(v.x, t.x, acc.x);
        acc.x = fma(-v.y, t.y, acc.x);
        acc.y = fma(v.x, t.y, acc.y);
        acc.y = fma(v.y, t.x, acc.y);
    };
    const int b4 = (int)((4 * (int64_t)b) % S.G);
    int m = (int)(((int64_t)c * b) % S.G);  // k b mod G
    int k = c;
    for (; k + 12 < S.K; k += 16) {
        double2 v[4], t[4];
        #pragma unroll
        for (int u = 0; u < 4; ++u) {
            t[u] = tw[m];
            v[u] = src[(int64_t)(k + 4 * u) * S.inner];
            m += b4;
            if (m >= S.G) m -= S.G;
        }
        #pragma unroll
        for (int u = 0; u < 4; ++u) term(k + 4 * u, v[u], t[u]);
    }
    for (; k < S.K; k += 4) {
        term(k, src[(int64_t)k * S.inner], tw[m]);
        m += b4;
        if (m >= S.G) m -= S.G;
    }
    acc.x += quad_swap<0xB1>(acc.x);
    acc.y += quad_swap<0xB1>(acc.y);
    acc.x += quad_swap<0x4E>(acc.x);
    acc.y += quad_swap<0x4E>(acc.y);
    if (c != 0) return;
    if (S.moments) {  // Taylor coefficient of t^b -> b-th derivative: times b! / rho^b
        double f = 1.0;
        for (int j = 1; j <= b; ++j) f *= (double)j / S.rho;
        acc.x *= f;
        acc.y *= f;
    }
    if (S.final_stage && !S.density) {
        probs[S.out_off + lq] = acc.x * S.scale;
        if (lq == 0 && err) err[S.inst] = (*status) ? INFINITY : 0.0;
    } else if (S.final_stage) {  // density mode: R = (1/prod G) sum over the half grid, complex
        out[S.out_off + lq] = cmk(acc.x * S.scale, acc.y * S.scale);
        if (lq == 0 && err) err[S.inst] = (*status) ? INFINITY : 0.0;
    } else {
        out[S.out_off + lq] = acc;
    }
}

// The same axis pass for extents K <= kDftColsK: one thread per (o, i) column
// loads its K inputs once into registers and writes all Bout outputs (no
// per-output index arithmetic or instance search, loads and stores coalesced
// along i).  Used for every descriptor with a small extent.
template <int KMAX>
__global__ void __launch_bounds__(256) dft_cols(const DftStageDev *__restrict__ st, const int64_t *__restrict__ prefix,
                                                int n, int64_t total, const double2 *__restrict__ twpool,
                                                const double2 *__restrict__ in, double2 *__restrict__ out,
                                                double *__restrict__ probs, double *__restrict__ err,
                                                const int *__restrict__ status)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;
    const int e = find_job(prefix, n, q);
    const DftStageDev S = st[e];
    const int64_t lq = q - prefix[e];
    const int64_t i = lq % S.inner, o = lq / S.inner;
    const double2 *__restrict__ src = in + S.in_off + o * S.K * S.inner + i;
    const double2 *__restrict__ tw = twpool + S.tw_off;
    double2 v[KMAX];
    #pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        v[k] = k < S.K ? src[(int64_t)k * S.inner] : cmk(0.0, 0.0);
        if (S.final_stage && !S.density && !(k == 0 || 2 * k == S.G)) {
            v[k].x *= 2.0;
            v[k].y *= 2.0;
        }
    }
    const int64_t obase = S.out_off + o * S.Bout * S.inner + i;
    for (int b = 0; b < S.Bout; ++b) {
        double2 acc = cmk(0.0, 0.0);
        int m = 0;
        #pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            if (k < S.K) {
                acc = cfma(v[k], tw[m], acc);
                m += b;
                if (m >= S.G) m -= S.G;
            }
        }
        if (S.moments) {
            double f = 1.0;
            for (int j = 1; j <= b; ++j) f *= (double)j / S.rho;
            acc.x *= f;
            acc.y *= f;
        }
        const int64_t oi = obase + (int64_t)b * S.inner;
        if (S.final_stage && !S.density) probs[oi] = acc.x * S.scale;
        else if (S.final_stage) out[oi] = cmk(acc.x * S.scale, acc.y * S.scale);
        else out[oi] = acc;
    }
    if (S.final_stage && lq == 0 && err) err[S.inst] = (*status) ? INFINITY : 0.0;
}

// ---------------------------------------------------------------------------
// Density mode (heralded states, Sec. VII).
//
// The heralding and traced rows of each internal block are eliminated per
// grid point as for probabilities; the kept modes' rows of A (and the loop
// vector) form a border of 2 g_k (+ 1) rows whose trailing Schur complement
// T is written by the LU kernel.  With the border built as
//     H'' = [[H_HH, -H_HG, -X gamma_H], [-A_GH, A_GG, gamma_G], [-gamma_H^T, gamma_G^T, 0]],
// S'' = I - diag(d) H'' has T = I - H''_BB - Gamma^T S^-1 D X Gamma with
// Gamma = [A_HG | gamma_H], so the generating function of the kept modes'
// matrix elements at this point,
//     sum_{u,v} <v|rho_G(w)|u> x^u y^v / sqrt(u! v!)
//         = G_H(w) exp(l^T c + 1/2 c^T Q c),   c = (y, x),
// (the master theorem, Eq. lhaf_master, on the heralding block with the
// c-dependent loop vector gamma_H + A_HG c) has Q = I - T_GG, l = -T_Ggamma and
// G_H(w) = Pr(0) prod_blocks det(S)^-1/2 exp(E), E = (1 - T_gammagamma) / 2.
//
// density_expand: one workgroup per evaluated point.  The normalised
// coefficients b_s = sqrt(s!) [c^s] (G_H exp(l^T c + 1/2 c^T Q c)) -- which
// are the matrix elements themselves -- satisfy (from d/dc_i of the
// exponential)
//     sqrt(s_i) b_s = l_i b_{s - e_i} + sum_j Q_ij sqrt(s_j - delta_ij) b_{s - e_i - e_j}
// for any i with s_i > 0.  Taking i as the first non-zero position of s
// (positions v_1..v_g, u_1..u_g, the last fastest in memory), every term on
// the right has the same leading zeros and only positions j >= i matter
// (s_j = 0 for j < i); the elements with first non-zero position i and s_i = t
// depend only on s_i = t - 1, t - 2 and on later positions, so positions are
// filled from the last one back, t = 1..N in order, the (N+1)^(2g-1-i)
// elements of each (i, t) in parallel.  b_0 = G_H(w) c_k / 2 folds in the
// half-grid weight (see density_hermitize).  Values stay in LDS when they
// fit, else in the output table itself.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) density_expand(const InstDev *__restrict__ insts,
                                                      const int32_t *__restrict__ dinst,
                                                      const int64_t *__restrict__ dprefix, int nd, int64_t lds_values,
                                                      const BlockDev *__restrict__ blocks,
                                                      const int32_t *__restrict__ rbpool,
                                                      const double2 *__restrict__ contrib,
                                                      const double2 *__restrict__ tpool, double2 *__restrict__ logg,
                                                      double2 *__restrict__ table)
{
    extern __shared__ double2 s_vals[];
    __shared__ double2 s_Q[kMaxKeepVars][kMaxKeepVars];
    __shared__ double2 s_l[kMaxKeepVars];
    __shared__ double2 s_acc;
    const int tid = threadIdx.x;
    const int64_t item = blockIdx.x;
    const int j0 = find_job(dprefix, nd, item);
    const InstDev &I = insts[dinst[j0]];
    const int64_t lp = item - dprefix[j0];
    const int nv = I.nvar;
    const int64_t E = I.E;
    const int N1 = I.fock_n + 1;
    for (int e = tid; e < kMaxKeepVars * kMaxKeepVars; e += blockDim.x) s_Q[e / kMaxKeepVars][e % kMaxKeepVars] = cmk(0.0, 0.0);
    if (tid < kMaxKeepVars) s_l[tid] = cmk(0.0, 0.0);
    if (tid == 0) {
        double2 acc = cmk(I.logpr0_re, I.logpr0_im);
        const double2 *c = contrib + I.c_off + lp * I.nblocks;
        for (int b = 0; b < I.nblocks; ++b) {
            acc.x += c[b].x;
            acc.y += c[b].y;
            const BlockDev &B = blocks[I.first_block + b];
            if (B.nkeep && B.bordered) {  // E = (1 - T_gammagamma) / 2
                const int nt = B.nkeep + 1;
                const double2 tg = tpool[B.t_off + lp * nt * nt + (int64_t)B.nkeep * nt + B.nkeep];
                acc.x += 0.5 * (1.0 - tg.x);
                acc.y -= 0.5 * tg.y;
            }
        }
        s_acc = acc;
    }
    __syncthreads();
    // Q = I - T_GG and l = -T_Ggamma per block, symmetrised, at the blocks' variable positions
    for (int b = 0; b < I.nblocks; ++b) {
        const BlockDev &B = blocks[I.first_block + b];
        if (!B.nkeep) continue;
        const int nk = B.nkeep, nt = nk + B.bordered;
        const double2 *__restrict__ T = tpool + B.t_off + lp * nt * nt;
        const int32_t *__restrict__ kv = rbpool + B.kv_off;
        for (int e = tid; e < nk * nk; e += blockDim.x) {
            const int a = e / nk, c = e % nk;
            const double2 t1 = T[a * nt + c], t2 = T[c * nt + a];
            s_Q[kv[a]][kv[c]] = cmk((a == c ? 1.0 : 0.0) - 0.5 * (t1.x + t2.x), -0.5 * (t1.y + t2.y));
        }
        if (B.bordered)
            for (int a = tid; a < nk; a += blockDim.x) {
                const double2 t1 = T[a * nt + nk], t2 = T[nk * nt + a];
                s_l[kv[a]] = cmk(-0.5 * (t1.x + t2.x), -0.5 * (t1.y + t2.y));
            }
    }
    double2 *__restrict__ gout = table + I.gv_off + lp * E;
    double2 *__restrict__ buf = E <= lds_values ? s_vals : gout;
    if (tid == 0) {
        const double2 acc = s_acc;
        logg[I.pt_off + lp] = acc;
        const int k1 = point_k(I, lp, 0);
        const double wk = (k1 == 0 || 2 * k1 == I.G[0]) ? 0.5 : 1.0;
        double sn, cs;
        sincos(acc.y, &sn, &cs);
        const double m = wk * exp(acc.x);
        buf[0] = cmk(m * cs, m * sn);
    }
    __syncthreads();
    int64_t st_i = 1;  // stride of position i: N1^(nv - 1 - i)
    for (int i = nv - 1; i >= 0; --i) {
        const double2 li = s_l[i];
        const double2 qii = s_Q[i][i];
        for (int t = 1; t < N1; ++t) {
            const double rt = 1.0 / sqrt((double)t);
            const double sq1 = sqrt((double)(t - 1));
            for (int64_t r = tid; r < st_i; r += blockDim.x) {
                const int64_t e = t * st_i + r;
                double2 acc = cmul(li, buf[e - st_i]);
                if (t >= 2) {
                    const double2 q = cmk(qii.x * sq1, qii.y * sq1);
                    acc = cfma(q, buf[e - 2 * st_i], acc);
                }
                int64_t rr = r, st_j = 1;
                for (int jj = nv - 1; jj > i; --jj) {
                    const int sj = (int)(rr % N1);
                    rr /= N1;
                    if (sj) {
                        const double f = sqrt((double)sj);
                        const double2 q = s_Q[i][jj];
                        acc = cfma(cmk(q.x * f, q.y * f), buf[e - st_i - st_j], acc);
                    }
                    st_j *= N1;
                }
                buf[e] = cmk(acc.x * rt, acc.y * rt);
            }
            __syncthreads();
        }
        st_i *= N1;
    }
    if (buf != gout)
        for (int64_t e = tid; e < E; e += blockDim.x) gout[e] = s_vals[e];
}

// rho(b~) = R + R^H per heralding pattern, with R the inverse DFT over the
// half grid (weights c_k / 2): the points w and conj(w) carry conjugate
// transposes of each other, rho_G(conj w) = rho_G(w)^H.  One workgroup per
// (instance, b~) matrix; R is in the buffer the instance's last DFT stage
// wrote, staged through LDS when it fits so that the transposed reads stay
// on chip.
__global__ void __launch_bounds__(256) density_hermitize(const InstDev *__restrict__ insts,
                                                         const int32_t *__restrict__ dinst,
                                                         const int64_t *__restrict__ mprefix, int nd,
                                                         int64_t lds_values, const double2 *__restrict__ bufA,
                                                         const double2 *__restrict__ bufB, double *__restrict__ out)
{
    extern __shared__ double2 s_vals[];
    const int64_t item = blockIdx.x;
    const int j0 = find_job(mprefix, nd, item);
    const InstDev &I = insts[dinst[j0]];
    const int64_t b = item - mprefix[j0];
    const int64_t E = I.E;
    int64_t D = 1;
    for (int k = 0; k < I.nvar / 2; ++k) D *= I.fock_n + 1;
    // stage s (0-based) writes bufB when s is even; the last stage of an instance is s = L - 1
    const double2 *__restrict__ R = ((I.L - 1) % 2 == 0 ? bufB : bufA) + I.gv_off + b * E;
    double2 *__restrict__ o = (double2 *)(out + I.prob_off) + b * E;
    const bool lds = E <= lds_values;
    if (lds) {
        for (int64_t e = threadIdx.x; e < E; e += blockDim.x) s_vals[e] = R[e];
        __syncthreads();
    }
    const double2 *__restrict__ src = lds ? s_vals : R;
    for (int64_t e = threadIdx.x; e < E; e += blockDim.x) {
        const int64_t v = e / D, u = e - v * D;
        const double2 x = src[e], y = src[u * D + v];
        o[e] = cmk(x.x + y.x, x.y - y.y);
    }
}

// ---------------------------------------------------------------------------
// Adjoint.  For a real loss L of the probabilities, with Ghat_k the adjoint
// DFT of dL/dP at grid point k and c_k the half-grid weight,
//     dL = Re sum_k omega_k d log G_k,   omega_k = c_k G_k Ghat_k.
// Per internal block, with S = I - D H and the bordered S' = [[S, D X gamma],
// [gamma^T, 1]] (whose inverse is Q, p = 1/Q_nn):
//     d log G = tr(W dH) + g^T d gamma + d log Pr(0),
//     W = 1/2 (Q_11 + (p^2 - p) Q_{:,n} Q_{n,:}) D,   g = -p/2 (Q_{:,n} + X D Q_{n,:}^T)
// (d log det S = tr(S^-1 dS); without displacement W = 1/2 S^-1 D, g = 0).
// lu_adjoint inverts S' in registers by Gauss-Jordan elimination without
// pivoting (same pivots as the LU, all in the right half-plane), over a chunk
// of grid points of one block, and accumulates omega W, omega g and omega.
// ---------------------------------------------------------------------------
template <int PR, int PC, int TR, int TC>
__global__ void __launch_bounds__(PR *PC)
lu_adjoint(const AdjArgs A)
{
    constexpr int NT = PR * PC;
    constexpr int N = PR * TR;
    static_assert(PR * TR == PC * TC, "square padding");
    static_assert(PC % PR == 0, "column owner must be uniform over a register row");
    __shared__ double2 s_u[2][N];
    __shared__ double2 s_l[2][N];
    __shared__ double2 s_d[N];
    __shared__ double2 s_qc[N];   // column n of Q (bordered)
    __shared__ double2 s_qr[N];   // row n of Q
    __shared__ double2 s_w[kMaxBins];
    __shared__ double2 s_om;

    const int tid = threadIdx.x;
    const int tx = tid % PC, ty = tid / PC;
    const int item = A.item_base + (int)blockIdx.x;  // absolute item index
    const int job = find_job(A.job_prefix, A.njobs, item);
    const int gbi = A.job_block[job];
    const GradBlockDev GB = A.gblocks[gbi];
    const InstDev &I = A.insts[GB.inst];
    const int nb = GB.nb;
    const int n = nb - GB.bordered;  // order of S
    const int64_t p0 = (int64_t)(item - A.job_prefix[job]) * A.chunk;
    const int64_t p1 = p0 + A.chunk < I.npts ? p0 + A.chunk : I.npts;
    const double2 *__restrict__ H = A.pool + GB.h_off;
    int64_t stride0 = 1;
    for (int l = 1; l < I.L; ++l) stride0 *= I.G[l];

    double2 z[TR][TC];
    double2 zg[TR];
    #pragma unroll
    for (int r = 0; r < TR; ++r) {
        zg[r] = cmk(0.0, 0.0);
        #pragma unroll
        for (int c = 0; c < TC; ++c) z[r][c] = cmk(0.0, 0.0);
    }
    double2 z0 = cmk(0.0, 0.0);

    for (int64_t pt = p0; pt < p1; ++pt) {
        __syncthreads();
        if (tid < I.L) point_w(I, pt, tid, s_w[tid]);
        if (tid == 0) {
            const double2 lg = A.logg[I.pt_off + pt];
            const double2 gh = A.ghat[I.pt_off + pt];
            const int64_t k1 = pt / stride0;
            const double ck = (k1 == 0 || 2 * k1 == I.G[0]) ? 1.0 : 2.0;
            double sn, cs;
            sincos(lg.y, &sn, &cs);
            const double m = ck * exp(lg.x);
            const double2 g = cmk(m * cs, m * sn);
            s_om = cmul(g, gh);
        }
        __syncthreads();
        for (int i = tid; i < nb; i += NT) {
            const int b = A.rbpool[GB.rb_off + i];
            s_d[i] = b < 0 ? cmk(1.0, 0.0) : s_w[b];
        }
        __syncthreads();
        const double2 om = s_om;

        double2 a[TR][TC];
        #pragma unroll
        for (int r = 0; r < TR; ++r) {
            const int i = r * PR + ty;
            #pragma unroll
            for (int c = 0; c < TC; ++c) {
                const int j = c * PC + tx;
                double2 v = cmk(i == j ? 1.0 : 0.0, 0.0);
                if (i < nb && j < nb) {
                    const double2 h = H[(int64_t)i * nb + j];
                    const double2 d = s_d[i];
                    v.x -= d.x * h.x - d.y * h.y;
                    v.y -= d.x * h.y + d.y * h.x;
                }
                a[r][c] = v;
            }
        }
        // Gauss-Jordan inversion in place: a <- S'^-1
        #pragma unroll
        for (int r = 0; r < TR; ++r) {
            const int cown = (r * PR) / PC;
            int kend = nb - r * PR;
            kend = kend < 0 ? 0 : (kend > PR ? PR : kend);
            for (int kk = 0; kk < kend; ++kk) {
                const int k = r * PR + kk;
                const int buf = k & 1;
                if (ty == kk) {
                    #pragma unroll
                    for (int c = 0; c < TC; ++c) s_u[buf][c * PC + tx] = a[r][c];
                }
                if (tx == k % PC) {
                    #pragma unroll
                    for (int r2 = 0; r2 < TR; ++r2) s_l[buf][r2 * PR + ty] = a[r2][cown];
                }
                __syncthreads();
                const double2 pinv = cinv(s_u[buf][k]);
                double2 u[TC];
                #pragma unroll
                for (int c = 0; c < TC; ++c) u[c] = cmul(s_u[buf][c * PC + tx], pinv);  // a_kj / p
                #pragma unroll
                for (int r2 = 0; r2 < TR; ++r2) {
                    const int i = r2 * PR + ty;
                    const double2 l = s_l[buf][i];  // a_ik
                    #pragma unroll
                    for (int c = 0; c < TC; ++c) {
                        const int j = c * PC + tx;
                        double2 v = cfnms(a[r2][c], l, u[c]);                 // a_ij - a_ik a_kj / p
                        if (r2 == r && i == k) v = u[c];                       // row k: a_kj / p
                        if (c == cown && j == k) v = cmk(-(l.x * pinv.x - l.y * pinv.y),
                                                         -(l.x * pinv.y + l.y * pinv.x));  // column k: -a_ik / p
                        if (r2 == r && c == cown && i == k && j == k) v = pinv;  // pivot: 1 / p
                        a[r2][c] = v;
                    }
                }
            }
        }
        // accumulate omega W (and omega g, omega)
        if (GB.bordered) {
            __syncthreads();
            #pragma unroll
            for (int r = 0; r < TR; ++r)
                #pragma unroll
                for (int c = 0; c < TC; ++c) {
                    const int i = r * PR + ty, j = c * PC + tx;
                    if (j == n && i < nb) s_qc[i] = a[r][c];
                    if (i == n && j < nb) s_qr[j] = a[r][c];
                }
            __syncthreads();
        }
        const double2 qnn = GB.bordered ? s_qc[n] : cmk(1.0, 0.0);
        const double2 pb = cinv(qnn);
        const double2 pp = cmk(pb.x * pb.x - pb.y * pb.y - pb.x, 2.0 * pb.x * pb.y - pb.y);  // p^2 - p
        #pragma unroll
        for (int r = 0; r < TR; ++r) {
            const int i = r * PR + ty;
            #pragma unroll
            for (int c = 0; c < TC; ++c) {
                const int j = c * PC + tx;
                if (i < n && j < n) {
                    double2 q = a[r][c];
                    if (GB.bordered) {
                        const double2 t = cmul(pp, cmul(s_qc[i], s_qr[j]));
                        q.x += t.x;
                        q.y += t.y;
                    }
                    const double2 w = cmul(cmk(0.5 * q.x, 0.5 * q.y), s_d[j]);
                    const double2 ow = cmul(om, w);
                    z[r][c].x += ow.x;
                    z[r][c].y += ow.y;
                }
            }
            if (GB.bordered && tx == 0 && i < n) {
                // g_i = -p/2 (Q_in + d_i' Q_ni'), i' the partner index in the other half
                const int half = n / 2;
                const int ip = i < half ? i + half : i - half;
                const double2 t = cmul(s_d[ip], s_qr[ip]);
                const double2 g = cmul(cmk(-0.5 * pb.x, -0.5 * pb.y), cmk(s_qc[i].x + t.x, s_qc[i].y + t.y));
                const double2 og = cmul(om, g);
                zg[r].x += og.x;
                zg[r].y += og.y;
            }
        }
        if (tid == 0) {
            z0.x += om.x;
            z0.y += om.y;
        }
    }
    // write this chunk's partial sums: n x n, then n, then 1
    double2 *__restrict__ out = A.partial + (int64_t)item * A.part_stride;
    #pragma unroll
    for (int r = 0; r < TR; ++r) {
        const int i = r * PR + ty;
        #pragma unroll
        for (int c = 0; c < TC; ++c) {
            const int j = c * PC + tx;
            if (i < n && j < n) out[(int64_t)i * n + j] = z[r][c];
        }
        if (tx == 0 && i < n) out[(int64_t)n * n + i] = zg[r];
    }
    if (tid == 0) out[(int64_t)n * n + n] = z0;
}

// Adjoint for blocks of order above the register classes: the same per-point
// sums as lu_adjoint, with Q = S'^-1 formed by a blocked Gauss-Jordan
// inversion in a per-workgroup workspace in HBM, kPanel columns per step.
// With K the step's rows and columns and D = A_KK (its inverse by
// Gauss-Jordan in LDS),
//     A_KK <- D^-1,   A_Kj <- D^-1 A_Kj,   A_iK <- -A_iK D^-1,
//     A_ij <- A_ij - A_iK D^-1 A_Kj        (i, j outside K),
// which leaves S'^-1 in place after the last step (no pivoting: each D is a
// trailing Schur complement block of S', whose pivots are those of the LU).
// The weighted sums are added into the item's slot of the partials (each
// element always by the same thread).  Persistent: workgroups loop over items.
// ---------------------------------------------------------------------------
size_t adj_big_lds_bytes(int ldw) {
    return sizeof(double2) * ((size_t)ldw * kPanel + kPanel * 64 + kPanel * kPanel + (size_t)ldw);
}

__global__ void __launch_bounds__(kBigThreads) adj_big_f64(const AdjArgs A, int nitems)
{
    static_assert(kBigThreads == kPanel * kPanel, "one thread per element of the pivot block");
    extern __shared__ double2 s_dyn[];
    const int ldw = A.ldw;
    double2 *s_panel = s_dyn;                           // ldw x kPanel: the step's column panel, all rows
    double2 *s_utile = s_panel + (size_t)ldw * kPanel;  // kPanel x 64: a tile of the new row panel
    double2 *s_dinv = s_utile + kPanel * 64;            // kPanel x kPanel: D, then D^-1
    double2 *s_d = s_dinv + kPanel * kPanel;            // ldw: d(w) per row
    double2 *s_qc = s_panel;                            // after the inversion: column n of Q
    double2 *s_qr = s_panel + ldw;                      //                      row n of Q
    __shared__ double2 s_w[kMaxBins];
    __shared__ double2 s_om;

    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4;
    double2 *__restrict__ W = A.work + (size_t)blockIdx.x * ldw * ldw;

    for (int it_ = blockIdx.x; it_ < nitems; it_ += gridDim.x) {
        const int item = A.item_base + it_;
        const int job = find_job(A.job_prefix, A.njobs, item);
        const GradBlockDev GB = A.gblocks[A.job_block[job]];
        const InstDev &I = A.insts[GB.inst];
        const int nb = GB.nb;
        const int n = nb - GB.bordered;
        const int64_t p0 = (int64_t)(item - A.job_prefix[job]) * A.chunk;
        const int64_t p1 = p0 + A.chunk < I.npts ? p0 + A.chunk : I.npts;
        const double2 *__restrict__ H = A.pool + GB.h_off;
        double2 *__restrict__ out = A.partial + (int64_t)item * A.part_stride;
        const int64_t nout = (int64_t)n * n + n + 1;
        int64_t stride0 = 1;
        for (int l = 1; l < I.L; ++l) stride0 *= I.G[l];
        __syncthreads();  // the previous item's last reads are done
        for (int64_t e = tid; e < nout; e += kBigThreads) out[e] = cmk(0.0, 0.0);

        for (int64_t pt = p0; pt < p1; ++pt) {
            __syncthreads();
            if (tid < I.L) point_w(I, pt, tid, s_w[tid]);
            if (tid == 0) {
                const double2 lg = A.logg[I.pt_off + pt];
                const double2 gh = A.ghat[I.pt_off + pt];
                const int64_t k1 = pt / stride0;
                const double ck = (k1 == 0 || 2 * k1 == I.G[0]) ? 1.0 : 2.0;
                double sn, cs;
                sincos(lg.y, &sn, &cs);
                const double m = ck * exp(lg.x);
                s_om = cmul(cmk(m * cs, m * sn), gh);
            }
            __syncthreads();
            for (int i = tid; i < nb; i += kBigThreads) {
                const int b = A.rbpool[GB.rb_off + i];
                s_d[i] = b < 0 ? cmk(1.0, 0.0) : s_w[b];
            }
            __syncthreads();
            const double2 om = s_om;
            for (int64_t e = tid; e < (int64_t)nb * nb; e += kBigThreads) {
                const int i = (int)(e / nb), j = (int)(e - (int64_t)i * nb);
                const double2 h = H[e];
                const double2 d = s_d[i];
                double2 v = cmk(i == j ? 1.0 : 0.0, 0.0);
                v.x -= d.x * h.x - d.y * h.y;
                v.y -= d.x * h.y + d.y * h.x;
                W[(size_t)i * ldw + j] = v;
            }
            __syncthreads();

            for (int k0 = 0; k0 < nb; k0 += kPanel) {
                const int kb = min(kPanel, nb - k0);
                for (int e = tid; e < nb * kPanel; e += kBigThreads) {
                    const int i = e / kPanel, t = e - i * kPanel;
                    s_panel[e] = t < kb ? W[(size_t)i * ldw + k0 + t] : cmk(0.0, 0.0);
                }
                __syncthreads();
                // D^-1 in LDS, one element per thread (identity outside kb x kb)
                const int r = tid / kPanel, c = tid - (tid / kPanel) * kPanel;
                s_dinv[tid] = (r < kb && c < kb) ? s_panel[(size_t)(k0 + r) * kPanel + c]
                                                 : cmk(r == c ? 1.0 : 0.0, 0.0);
                __syncthreads();
                for (int kk = 0; kk < kb; ++kk) {
                    const double2 pinv = cinv(s_dinv[kk * kPanel + kk]);
                    const double2 a_rk = s_dinv[r * kPanel + kk];
                    const double2 a_kc = s_dinv[kk * kPanel + c];
                    const double2 a_rc = s_dinv[tid];
                    __syncthreads();
                    const double2 u = cmul(a_kc, pinv);
                    double2 v;
                    if (r == kk && c == kk) v = pinv;
                    else if (r == kk) v = u;
                    else if (c == kk) v = cmk(-(a_rk.x * pinv.x - a_rk.y * pinv.y), -(a_rk.x * pinv.y + a_rk.y * pinv.x));
                    else v = cfnms(a_rc, a_rk, u);
                    s_dinv[tid] = v;
                    __syncthreads();
                }
                // row panel: A_Kj <- D^-1 A_Kj, one column j outside K per thread
                for (int j = tid; j < nb; j += kBigThreads) {
                    if (j >= k0 && j < k0 + kb) continue;
                    double2 x[kPanel];
                    #pragma unroll
                    for (int t = 0; t < kPanel; ++t) x[t] = t < kb ? W[(size_t)(k0 + t) * ldw + j] : cmk(0.0, 0.0);
                    #pragma unroll
                    for (int t = 0; t < kPanel; ++t) {
                        if (t >= kb) break;
                        double2 y = cmk(0.0, 0.0);
                        #pragma unroll
                        for (int s2 = 0; s2 < kPanel; ++s2) y = cfma(s_dinv[t * kPanel + s2], x[s2], y);
                        W[(size_t)(k0 + t) * ldw + j] = y;
                    }
                }
                __syncthreads();
                // A_ij -= C_i (D^-1 A_Kj) for every i, j outside K, in 64 x 64 tiles
                for (int jt = 0; jt < nb; jt += 64) {
                    for (int e = tid; e < kPanel * 64; e += kBigThreads) {
                        const int t = e / 64, jj = jt + (e - (e / 64) * 64);
                        const bool ok = t < kb && jj < nb && (jj < k0 || jj >= k0 + kb);
                        s_utile[e] = ok ? W[(size_t)(k0 + t) * ldw + jj] : cmk(0.0, 0.0);
                    }
                    __syncthreads();
                    for (int it = 0; it < nb; it += 64) {
                        double2 acc[4][4];
                        #pragma unroll
                        for (int a = 0; a < 4; ++a)
                            #pragma unroll
                            for (int b = 0; b < 4; ++b) {
                                const int i = it + ty + 16 * a, j = jt + tx + 16 * b;
                                acc[a][b] = (i < nb && j < nb) ? W[(size_t)i * ldw + j] : cmk(0.0, 0.0);
                            }
                        for (int t = 0; t < kb; ++t) {
                            double2 l[4], u[4];
                            #pragma unroll
                            for (int a = 0; a < 4; ++a) {
                                const int i = it + ty + 16 * a;
                                l[a] = (i < nb && (i < k0 || i >= k0 + kb)) ? s_panel[(size_t)i * kPanel + t]
                                                                            : cmk(0.0, 0.0);
                            }
                            #pragma unroll
                            for (int b = 0; b < 4; ++b) u[b] = s_utile[t * 64 + tx + 16 * b];
                            #pragma unroll
                            for (int a = 0; a < 4; ++a)
                                #pragma unroll
                                for (int b = 0; b < 4; ++b) acc[a][b] = cfnms(acc[a][b], l[a], u[b]);
                        }
                        #pragma unroll
                        for (int a = 0; a < 4; ++a)
                            #pragma unroll
                            for (int b = 0; b < 4; ++b) {
                                const int i = it + ty + 16 * a, j = jt + tx + 16 * b;
                                if (i < nb && j < nb && (i < k0 || i >= k0 + kb) && (j < k0 || j >= k0 + kb))
                                    W[(size_t)i * ldw + j] = acc[a][b];
                            }
                    }
                    __syncthreads();
                }
                // column panel: A_iK <- -C_i D^-1 outside K, and D^-1 on K
                for (int e = tid; e < nb * kPanel; e += kBigThreads) {
                    const int i = e / kPanel, cc = e - i * kPanel;
                    if (cc >= kb) continue;
                    double2 v;
                    if (i >= k0 && i < k0 + kb) {
                        v = s_dinv[(i - k0) * kPanel + cc];
                    } else {
                        double2 y = cmk(0.0, 0.0);
                        for (int s2 = 0; s2 < kb; ++s2) y = cfma(s_panel[(size_t)i * kPanel + s2], s_dinv[s2 * kPanel + cc], y);
                        v = cmk(-y.x, -y.y);
                    }
                    W[(size_t)i * ldw + k0 + cc] = v;
                }
                __syncthreads();
            }

            // accumulate omega W, omega g, omega (as lu_adjoint)
            if (GB.bordered)
                for (int i = tid; i < nb; i += kBigThreads) {
                    s_qc[i] = W[(size_t)i * ldw + n];
                    s_qr[i] = W[(size_t)n * ldw + i];
                }
            __syncthreads();
            const double2 qnn = GB.bordered ? s_qc[n] : cmk(1.0, 0.0);
            const double2 pb = cinv(qnn);
            const double2 pp = cmk(pb.x * pb.x - pb.y * pb.y - pb.x, 2.0 * pb.x * pb.y - pb.y);  // p^2 - p
            for (int64_t e = tid; e < (int64_t)n * n; e += kBigThreads) {
                const int i = (int)(e / n), j = (int)(e - (int64_t)i * n);
                double2 q = W[(size_t)i * ldw + j];
                if (GB.bordered) {
                    const double2 t = cmul(pp, cmul(s_qc[i], s_qr[j]));
                    q.x += t.x;
                    q.y += t.y;
                }
                const double2 ow = cmul(om, cmul(cmk(0.5 * q.x, 0.5 * q.y), s_d[j]));
                out[e].x += ow.x;
                out[e].y += ow.y;
            }
            if (GB.bordered) {
                const int half = n / 2;
                for (int i = tid; i < n; i += kBigThreads) {
                    const int ip = i < half ? i + half : i - half;
                    const double2 t = cmul(s_d[ip], s_qr[ip]);
                    const double2 g = cmul(cmk(-0.5 * pb.x, -0.5 * pb.y), cmk(s_qc[i].x + t.x, s_qc[i].y + t.y));
                    const double2 og = cmul(om, g);
                    out[(int64_t)n * n + i].x += og.x;
                    out[(int64_t)n * n + i].y += og.y;
                }
            }
            if (tid == 0) {
                out[(int64_t)n * n + n].x += om.x;
                out[(int64_t)n * n + n].y += om.y;
            }
        }
    }
}

// Sum the chunk partials of every gradient block in a fixed order.
__global__ void adjoint_reduce(const GradBlockDev *__restrict__ gblocks, const int64_t *__restrict__ elem_prefix,
                               int ngb, int64_t total, const double2 *__restrict__ partial, int64_t part_stride,
                               double2 *__restrict__ zout)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const int b = find_job(elem_prefix, ngb, e);
    const GradBlockDev GB = gblocks[b];
    const int64_t le = e - elem_prefix[b];
    double2 acc = cmk(0.0, 0.0);
    for (int c = 0; c < GB.nchunks; ++c) {
        const double2 v = partial[(int64_t)(GB.first_item + c) * part_stride + le];
        acc.x += v.x;
        acc.y += v.y;
    }
    zout[GB.z_off + le] = acc;
}

// Move each instance's adjoint-DFT result (ping-pong buffer chosen by the
// parity of its number of axes) to the point-indexed buffer.
__global__ void adjoint_gather(const InstDev *__restrict__ insts, const int64_t *__restrict__ inst_pt_prefix,
                               int n_inst, int64_t npts, const int64_t *__restrict__ buf_off,
                               const double2 *__restrict__ bufA, const double2 *__restrict__ bufB,
                               double2 *__restrict__ ghat)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npts) return;
    const int i = find_job(inst_pt_prefix, n_inst, p);
    const InstDev &I = insts[i];
    const double2 *src = (I.L & 1) ? bufB : bufA;
    ghat[p] = src[buf_off[i] + (p - I.pt_off)];
}

// Real dL/dP -> complex buffer scaled by 1/prod G (input of the adjoint DFT).
__global__ void adjoint_seed(const InstDev *__restrict__ insts, const int64_t *__restrict__ prob_prefix, int n_inst,
                             int64_t nprobs, const double *__restrict__ dprobs, const int64_t *__restrict__ buf_off,
                             double2 *__restrict__ out)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nprobs) return;
    const int i = find_job(prob_prefix, n_inst, q);
    const InstDev &I = insts[i];
    double gprod = 1;
    for (int l = 0; l < I.L; ++l) gprod *= I.G[l];
    out[buf_off[i] + (q - I.prob_off)] = cmk(dprobs[q] / gprod, 0.0);
}

// ---------------------------------------------------------------------------
// Mixed path.  After the FP32 pass, the value of G at point k carries a
// relative error of at most tau (per instance); it enters every probability as
// c_k |G_k| tau / prod G (c_k = 1 or 2 on the half grid), so the points left in
// FP32 add at most (tau / prod G) sum_{k in FP32} c_k |G_k| to any
// probability.  The points are ranked by |G_k| in buckets of a quarter octave
// (bucket b holds 2^-(b+1)/4 < |G| <= 2^-b/4, the last one everything
// smaller); the FP32 set is the longest run of buckets, from the smallest |G|
// up, whose summed c_k |G_k| stays within the budget tol prod G / tau.  The
// sums are taken in fixed point (units of 2^-28, rounded up, 64-bit integer
// atomics), so the cut does not depend on the order of the additions and the
// true sum of the FP32 set is at most the budget.  Every other point is
// factorised again in FP64; mixed_err then reports the exact bound of what is
// left in FP32.
// ---------------------------------------------------------------------------
__global__ void zero_ints(int *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void zero_u64(unsigned long long *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

constexpr double kMixedScale = 268435456.0;  // 2^28: fixed-point unit of the bucket sums

// bucket of a point from its FP32 log G (NaN lands in bucket 0: always redone)
__device__ __forceinline__ int mixed_bucket(double logg_re) {
    const double b = -logg_re * (kMixedBucketsPerOctave * 1.4426950408889634);  // 1 / ln 2
    if (!(b > 0.0)) return 0;
    return b >= (double)(kMixedBuckets - 1) ? kMixedBuckets - 1 : (int)b;
}

__device__ __forceinline__ double half_grid_weight(const InstDev &I, int64_t lp) {
    int64_t stride = 1;
    for (int l = 1; l < I.L; ++l) stride *= I.G[l];
    const int64_t k1 = lp / stride;
    return (k1 == 0 || 2 * k1 == I.G[0]) ? 1.0 : 2.0;
}

// hist[i * kMixedBuckets + b] += ceil(c_k |G_k| 2^28) over the points of
// instance i with an FP32 block
__global__ void mixed_hist(const InstDev *__restrict__ insts, const int64_t *__restrict__ inst_pt_prefix,
                           int n_inst, int64_t npts, const double2 *__restrict__ logg,
                           unsigned long long *__restrict__ hist)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npts) return;
    const int i = find_job(inst_pt_prefix, n_inst, p);
    const InstDev &I = insts[i];
    if (!(I.tau > 0.0)) return;
    const double lg = logg[p].x;
    const double g = exp(fmin(lg, 1.0));  // |G| <= 1 up to rounding; NaN stays NaN
    const double wgt = half_grid_weight(I, p - I.pt_off) * g * kMixedScale;
    const unsigned long long q = isfinite(wgt) ? (unsigned long long)ceil(wgt) : (1ull << 40);
    atomicAdd(&hist[(int64_t)i * kMixedBuckets + mixed_bucket(lg)], q);
}

// one wave per instance: cut[i] = largest bucket index that is factorised
// again (-1: none), scanning from the smallest |G| up
__global__ void mixed_cut(const InstDev *__restrict__ insts, int n_inst, double tol,
                          const unsigned long long *__restrict__ hist, int *__restrict__ cut)
{
    const int i = blockIdx.x;
    if (i >= n_inst || threadIdx.x != 0) return;
    const InstDev &I = insts[i];
    if (!(I.tau > 0.0)) {
        cut[i] = -1;
        return;
    }
    double gprod = 1;
    for (int l = 0; l < I.L; ++l) gprod *= I.G[l];
    const double bd = floor(tol * gprod / I.tau * kMixedScale);
    const unsigned long long budget = bd >= 4.0e18 ? 4000000000000000000ull : (unsigned long long)bd;
    const unsigned long long *h = hist + (int64_t)i * kMixedBuckets;
    unsigned long long acc = 0;
    int b = kMixedBuckets - 1;
    for (; b >= 0; --b) {
        acc += h[b];
        if (acc > budget) break;
    }
    cut[i] = b;  // buckets above b stay in FP32
}

__global__ void select_points(const InstDev *__restrict__ insts, const int64_t *__restrict__ inst_pt_prefix,
                              int n_inst, int64_t npts, const BlockDev *__restrict__ blocks,
                              const double2 *__restrict__ logg, const int *__restrict__ cut,
                              int2 *__restrict__ list_base, const int64_t *__restrict__ list_off,
                              int *__restrict__ counts, int n_lists)
{
    // every lane takes part in the ballots below: no early return
    const int lane = threadIdx.x & 63;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int nb = 0, first = 0;
    int64_t lp = 0;
    if (p < npts) {
        const int i = find_job(inst_pt_prefix, n_inst, p);
        const InstDev &I = insts[i];
        if (I.tau > 0.0 && mixed_bucket(logg[p].x) <= cut[i]) {
            nb = I.nblocks;
            first = I.first_block;
            lp = p - I.pt_off;
        }
    }
    for (int b = 0; __any(b < nb); ++b) {
        int cls = -1;
        if (b < nb) {
            const BlockDev &B = blocks[first + b];
            if (B.fp32 && B.cls >= 0 && B.cls < n_lists && list_off[B.cls] >= 0) cls = B.cls;
        }
        // one atomic per wave and list: lanes of the same list share it
        unsigned long long pending = __ballot(cls >= 0);
        while (pending) {
            const int leader = __ffsll(pending) - 1;
            const int c = __shfl(cls, leader);
            const unsigned long long grp = __ballot(cls == c);
            int base = 0;
            if (lane == leader) base = atomicAdd(&counts[c], __popcll(grp));
            base = __shfl(base, leader);
            if (cls == c)
                list_base[list_off[c] + base + __popcll(grp & ((1ull << lane) - 1))] = make_int2(first + b, (int)lp);
            pending &= ~grp;
        }
    }
}

// Per instance: (1 / prod G) sum over the points left in FP32 of c_k |G_k| tau,
// the bound on the error of every probability (deterministic order).
__global__ void mixed_err(const InstDev *__restrict__ insts, const double2 *__restrict__ logg,
                          const int *__restrict__ cut, double *__restrict__ err, const int *__restrict__ status)
{
    __shared__ double2 s_red[256 / 64 + 1];
    const InstDev &I = insts[blockIdx.x];
    const int ci = cut[blockIdx.x];
    double acc = 0.0;
    if (I.tau > 0.0)
        for (int64_t p = threadIdx.x; p < I.npts; p += blockDim.x) {
            const double lg = logg[I.pt_off + p].x;
            if (mixed_bucket(lg) <= ci) continue;
            acc += half_grid_weight(I, p) * exp(lg);
        }
    double2 t = block_sum<256>(cmk(acc, 0.0), s_red);
    if (threadIdx.x == 0) {
        double gprod = 1;
        for (int l = 0; l < I.L; ++l) gprod *= I.G[l];
        err[blockIdx.x] = (*status) ? INFINITY : t.x * I.tau / gprod;
    }
}

template <int PR, int PC, int TR, int TC>
static hipError_t launch_reg(const LuLaunch &a, hipStream_t st) {
    LuArgs A{a.job_block, a.job_prefix, a.njobs, a.nitems, a.list, a.list_count, a.blocks, a.insts, a.pool,
             a.rbpool, a.eigpool, a.contrib, a.status, a.tpool, a.tw, a.job_hint};
    // one item per workgroup; for a device-built list the grid covers its capacity and
    // workgroups past the list's length return at once
    const int64_t grid = a.list ? a.list_capacity : a.nitems;
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL((lu_reg<double, PR, PC, TR, TC>), dim3((unsigned)grid), dim3(PR * PC), 0, st, A);
    return hipGetLastError();
}

int reg_class_limit(int cls) {
    switch (cls) {
        case 0: return 32;
        case 1: return 64;
        case 2: return 96;
        case 3: return 128;
        case 4: return 144;
        default: return 0;
    }
}

// thread-grid shapes <PR, PC, TR, TC> per register class (the autotuner picks one)
// FP64 kernel shapes per register class (the autotuner picks one): the
// register kernel's thread grids <PR, PC, TR, TC>, then (classes 0..2) FP64
// MFMA wave layouts <NTILE, WR, WC, OCC>.  Variant 0 is the default; blocks
// with kept modes (density mode) need a register-kernel shape
// (reg_kernel_variants), which writes the trailing Schur complement.
static constexpr int kRegShapes[kRegClasses] = {2, 3, 2, 1, 1};
static constexpr int kMfma64Shapes[kRegClasses] = {3, 3, 3, 0, 0};
int reg_variants(int cls) { return cls >= 0 && cls < kRegClasses ? kRegShapes[cls] + kMfma64Shapes[cls] : 0; }
int reg_kernel_variants(int cls) { return cls >= 0 && cls < kRegClasses ? kRegShapes[cls] : 0; }

const char *reg_variant_name(int cls, int v) {
    static const char *names[kRegClasses][6] = {
        {"lu_reg<double,8,8,4,4>", "lu_reg<double,8,16,4,2>", "lu_mfma_f64<2,1,1>", "lu_mfma_f64<2,1,2>",
         "lu_mfma_f64<2,1,1,3>"},
        {"lu_reg<double,16,16,4,4>", "lu_reg<double,8,16,8,4>", "lu_reg<double,16,32,4,2>", "lu_mfma_f64<4,2,2>",
         "lu_mfma_f64<4,1,2>", "lu_mfma_f64<4,2,2,3>"},
        {"lu_reg<double,16,32,6,3>", "lu_reg<double,16,16,6,6>", "lu_mfma_f64<6,2,2>", "lu_mfma_f64<6,2,4>",
         "lu_mfma_f64<6,3,2>"},
        {"lu_reg<double,16,32,8,4>"},
        {"lu_reg<double,16,48,9,3>"}};
    return (cls >= 0 && cls < kRegClasses && v >= 0 && v < reg_variants(cls)) ? names[cls][v] : "";
}

template <int NTILE, int WR, int WC, int OCC = 1>
static hipError_t launch_mfma64(const LuLaunch &a, hipStream_t st);

hipError_t launch_lu_reg(int cls, int v, const LuLaunch &a, hipStream_t st) {
    if (!a.list && a.nitems <= 0) return hipSuccess;
    switch (cls * 8 + v) {
        case 0: return launch_reg<8, 8, 4, 4>(a, st);
        case 1: return launch_reg<8, 16, 4, 2>(a, st);
        case 2: return launch_mfma64<2, 1, 1>(a, st);
        case 3: return launch_mfma64<2, 1, 2>(a, st);
        case 4: return launch_mfma64<2, 1, 1, 3>(a, st);
        case 8: return launch_reg<16, 16, 4, 4>(a, st);
        case 9: return launch_reg<8, 16, 8, 4>(a, st);
        case 10: return launch_reg<16, 32, 4, 2>(a, st);
        case 11: return launch_mfma64<4, 2, 2>(a, st);
        case 12: return launch_mfma64<4, 1, 2>(a, st);
        case 13: return launch_mfma64<4, 2, 2, 3>(a, st);
        case 16: return launch_reg<16, 32, 6, 3>(a, st);
        case 17: return launch_reg<16, 16, 6, 6>(a, st);
        case 18: return launch_mfma64<6, 2, 2>(a, st);
        case 19: return launch_mfma64<6, 2, 4>(a, st);
        case 20: return launch_mfma64<6, 3, 2>(a, st);
        case 24: return launch_reg<16, 32, 8, 4>(a, st);
        case 32: return launch_reg<16, 48, 9, 3>(a, st);
        default: return hipErrorInvalidValue;
    }
}

template <int NTILE, int WR, int WC, int OCC = 1>
static hipError_t launch_mfma(const LuLaunch &a, hipStream_t st) {
    LuArgs A{a.job_block, a.job_prefix, a.njobs, a.nitems, a.list, a.list_count, a.blocks, a.insts, a.pool,
             a.rbpool, a.eigpool, a.contrib, a.status, a.tpool, a.tw, a.job_hint};
    const int64_t grid = a.list ? a.list_capacity : a.nitems;
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL((lu_mfma_f32<NTILE, WR, WC, OCC>), dim3((unsigned)grid), dim3(64 * WR * WC),
                       sizeof(MfmaLds<float, NTILE, WR, WC>), st, A);
    return hipGetLastError();
}

template <int NTILE, int WR, int WC, int OCC>
static hipError_t launch_mfma64(const LuLaunch &a, hipStream_t st) {
    LuArgs A{a.job_block, a.job_prefix, a.njobs, a.nitems, a.list, a.list_count, a.blocks, a.insts, a.pool,
             a.rbpool, a.eigpool, a.contrib, a.status, a.tpool, a.tw, a.job_hint};
    const int64_t grid = a.list ? a.list_capacity : a.nitems;
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL((lu_mfma_f64<NTILE, WR, WC, OCC>), dim3((unsigned)grid), dim3(64 * WR * WC),
                       sizeof(MfmaLds<double, NTILE, WR, WC>), st, A);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Kernel R: low-rank blocks (fully distinguishable inputs, App. D).  When H =
// V diag(lambda) V^H has rank r <= kLowRankMax, det(I - D H) = det(I_r - C)
// with C = G_t + sum_l w_l G_l (Sylvester), the r x r matrices G_g =
// diag(lambda) V^H E_g V coming from the host.  One thread per (block, point):
// C from (L + 1) r^2 complex multiply-adds, then the unpivoted LU of I_r - C
// in registers.  With s = sign(lambda), I_r - C is the diagonal similarity
// transform (by |lambda|^1/2) of I_r - s |lambda|^1/2 V^H D V |lambda|^1/2,
// whose second term has norm at most ||H|| max|w| < 1: it is accretive, and
// a diagonal similarity keeps every principal minor, so the pivots lie in the
// right half-plane and the sum of their principal logarithms is the
// continuous branch, exactly as for S itself.  Two pivots of the right
// half-plane have a product whose argument stays inside (-pi, pi), so the
// logarithms are taken pairwise.
//
// A workgroup takes 16 blocks of one instance and a run of kLrRun tiles of 16
// points: the blocks' G matrices and the run's values of w are staged in LDS
// once, then lane t takes block t mod 16 of point t / 16 of each tile, so that
// a wave writes four runs of 16 adjacent contribution slots and the chain of
// descriptor loads is paid once per 16 x 16 kLrRun items.
constexpr int kLrTile = 16;
constexpr int kLrRun = 8;

// N items of one block at a time (points w0 + n wstep), their elimination
// chains interleaved so that one lane has N independent FP64 chains in flight;
// items with on[n] false are computed on whatever their w holds and ignored.
template <int R, int N>
__device__ __forceinline__ void lowrank_logdets(const double2 *G, const double2 *w0, int wstep, int L,
                                                const bool (&on)[N], double2 (&acc)[N], bool &bad) {
    double2 m[N][R][R];
    #pragma unroll
    for (int a = 0; a < R; ++a)
        #pragma unroll
        for (int c = 0; c < R; ++c) {
            const double2 g = G[a * R + c];
            #pragma unroll
            for (int n = 0; n < N; ++n) m[n][a][c] = cmk((a == c ? 1.0 : 0.0) - g.x, -g.y);
        }
    for (int l = 0; l < L; ++l) {
        const double2 *Gl = G + (l + 1) * R * R;
        double2 wl[N];
        #pragma unroll
        for (int n = 0; n < N; ++n) wl[n] = w0[n * wstep + l];
        #pragma unroll
        for (int a = 0; a < R; ++a)
            #pragma unroll
            for (int c = 0; c < R; ++c) {
                const double2 g = Gl[a * R + c];
                #pragma unroll
                for (int n = 0; n < N; ++n) m[n][a][c] = cfnms(m[n][a][c], wl[n], g);
            }
    }
    double2 held[N];
    #pragma unroll
    for (int n = 0; n < N; ++n) {
        acc[n] = cmk(0.0, 0.0);
        held[n] = cmk(1.0, 0.0);
    }
    #pragma unroll
    for (int k = 0; k < R; ++k) {
        #pragma unroll
        for (int n = 0; n < N; ++n) {
            const double2 p = m[n][k][k];
            if (on[n] && (!(p.x > 0.0) || !isfinite(p.x) || !isfinite(p.y))) bad = true;
            if (k % 2 == 0) {
                held[n] = p;
            } else {
                const double2 q = clog(cmul(held[n], p));
                acc[n].x += q.x;
                acc[n].y += q.y;
            }
            if (k + 1 < R) {
                const double2 pinv = cinv(p);
                #pragma unroll
                for (int i = k + 1; i < R; ++i) {
                    const double2 li = cmul(m[n][i][k], pinv);
                    #pragma unroll
                    for (int j = k + 1; j < R; ++j) m[n][i][j] = cfnms(m[n][i][j], li, m[n][k][j]);
                }
            }
        }
    }
    if (R % 2 == 1) {
        #pragma unroll
        for (int n = 0; n < N; ++n) {
            const double2 q = clog(held[n]);
            acc[n].x += q.x;
            acc[n].y += q.y;
        }
    }
}

template <int R>
__global__ void __launch_bounds__(kLrTile * kLrTile)
lowrank_points(const int2 *__restrict__ jobs, const int64_t *__restrict__ prefix, int njobs,
               const int32_t *__restrict__ lrblk, const BlockDev *__restrict__ blocks,
               const InstDev *__restrict__ insts, const double2 *__restrict__ pool,
               const double2 *__restrict__ tw, double2 *__restrict__ contrib, int *__restrict__ status,
               int gstride, int wstride) {
    extern __shared__ double2 s_lr[];
    double2 *s_g = s_lr;                               // 16 blocks x gstride
    double2 *s_w = s_lr + kLrTile * gstride;           // kLrRun x 16 points x wstride
    // the tile (uniform over the workgroup): job j covers blocks lrblk[x .. x + y)
    // of one instance, its tiles ordered (point run, block tile)
    const int64_t tile = blockIdx.x;
    const int j = find_job(prefix, njobs, tile);
    const int2 jc = jobs[j];
    const int nbt = (jc.y + kLrTile - 1) / kLrTile;
    const int64_t local = tile - prefix[j];
    const int64_t p0 = (local / nbt) * (kLrTile * kLrRun);
    const int q0 = (int)(local % nbt) * kLrTile;
    const InstDev &I = insts[blocks[lrblk[jc.x]].inst];
    const int L = I.L;
    const int64_t npts = I.npts;
    const int t = threadIdx.x;
    {
        // 16 threads per block slot copy its (L + 1) r^2 matrices; then w of the run's points
        const int slot = t / kLrTile, e0 = t % kLrTile;
        if (q0 + slot < jc.y) {
            const BlockDev &B = blocks[lrblk[jc.x + q0 + slot]];
            const int n = (L + 1) * R * R;
            for (int e = e0; e < n; e += kLrTile) s_g[slot * gstride + e] = pool[B.lr_off + e];
        }
        for (int e = t; e < kLrTile * kLrRun * L; e += kLrTile * kLrTile) {
            const int ps = e / L, l = e - ps * L;
            if (p0 + ps < npts) point_w(I, p0 + ps, l, s_w[ps * wstride + l], tw);
        }
    }
    __syncthreads();
    const int qs = t % kLrTile;
    if (q0 + qs >= jc.y) return;
    const BlockDev &B = blocks[lrblk[jc.x + q0 + qs]];
    const int64_t slot_off = I.c_off + B.blk;
    const double2 *G = s_g + qs * gstride;
    bool bad = false;
    // points per pass, kLrTile apart: eight independent chains per lane for rank
    // <= 2 (62.8 us against 154.6 us with one on the 5.08M rank-2 items of the M = 144
    // distinguishable circuit), fewer for larger ranks to stay within the registers
    constexpr int N = R <= 2 ? 8 : (R == 3 ? 4 : 2);
    for (int ps = t / kLrTile; ps < kLrTile * kLrRun; ps += N * kLrTile) {
        bool on[N];
        #pragma unroll
        for (int n = 0; n < N; ++n) on[n] = p0 + ps + n * kLrTile < npts;
        if (!on[0]) break;
        double2 acc[N];
        lowrank_logdets<R, N>(G, s_w + ps * wstride, kLrTile * wstride, L, on, acc, bad);
        #pragma unroll
        for (int n = 0; n < N; ++n)
            if (on[n]) contrib[slot_off + (p0 + ps + n * kLrTile) * I.nblocks] = cmk(-0.5 * acc[n].x, -0.5 * acc[n].y);
    }
    if (bad) atomicOr(status, 1);
}

size_t lowrank_lds_bytes(int gstride, int wstride) {
    return sizeof(double2) * ((size_t)kLrTile * gstride + (size_t)kLrTile * kLrRun * wstride);
}
int lowrank_points_per_tile() { return kLrTile * kLrRun; }

hipError_t launch_lowrank_points(int r, const int2 *jobs, const int64_t *prefix, int njobs, int64_t ntiles,
                                 const int32_t *lrblk, const BlockDev *blocks, const InstDev *insts,
                                 const double2 *pool, const double2 *tw, double2 *contrib, int *status,
                                 int gstride, int wstride, hipStream_t st) {
    if (ntiles <= 0) return hipSuccess;
    if (r < 1 || r > kLowRankMax || njobs <= 0 || jobs == nullptr || prefix == nullptr || lrblk == nullptr ||
        ntiles > 0x7fffffff || gstride < 1 || gstride > (kMaxBins + 1) * r * r || wstride < 1 || wstride > kMaxBins)
        return hipErrorInvalidValue;
    const dim3 grid((unsigned)ntiles), block(kLrTile * kLrTile);
    const size_t lds = lowrank_lds_bytes(gstride, wstride);
    switch (r) {
        case 1: hipLaunchKernelGGL(lowrank_points<1>, grid, block, lds, st, jobs, prefix, njobs, lrblk, blocks, insts,
                                   pool, tw, contrib, status, gstride, wstride); break;
        case 2: hipLaunchKernelGGL(lowrank_points<2>, grid, block, lds, st, jobs, prefix, njobs, lrblk, blocks, insts,
                                   pool, tw, contrib, status, gstride, wstride); break;
        case 3: hipLaunchKernelGGL(lowrank_points<3>, grid, block, lds, st, jobs, prefix, njobs, lrblk, blocks, insts,
                                   pool, tw, contrib, status, gstride, wstride); break;
        default: hipLaunchKernelGGL(lowrank_points<4>, grid, block, lds, st, jobs, prefix, njobs, lrblk, blocks, insts,
                                    pool, tw, contrib, status, gstride, wstride); break;
    }
    return hipGetLastError();
}

hipError_t launch_lu_one_tile(const LuLaunch &a, hipStream_t st) {
    if (a.list || a.nitems <= 0) return a.list ? hipErrorInvalidValue : hipSuccess;
    return launch_mfma64<1, 1, 1>(a, st);
}

template <int NTILE, int WR, int WC, int OCC = 1>
static hipError_t prepare_mfma() {
    return hipFuncSetAttribute((const void *)lu_mfma_f32<NTILE, WR, WC, OCC>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)sizeof(MfmaLds<float, NTILE, WR, WC>));
}

template <int NTILE, int WR, int WC, int OCC = 1>
static hipError_t prepare_mfma64() {
    return hipFuncSetAttribute((const void *)lu_mfma_f64<NTILE, WR, WC, OCC>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)sizeof(MfmaLds<double, NTILE, WR, WC>));
}

int mfma_class_limit(int cls) {
    switch (cls) {
        case 0: return 32;
        case 1: return 64;
        case 2: return 96;
        case 3: return 128;
        case 4: return 144;
        case 5: return 192;
        default: return 0;
    }
}

// wave layouts <NTILE, WR, WC> per FP32 MFMA class (the autotuner picks one)
int mfma_variants(int cls) { return cls == 0 ? 3 : cls == 1 ? 8 : cls == 2 ? 5 : cls < kMfmaClasses ? 1 : 0; }

// <NTILE, WR, WC> or <NTILE, WR, WC, OCC> (register cap for OCC waves per SIMD);
// variant 0 is the default shape (CGD_FLAG_NO_AUTOTUNE) and wins ties
const char *mfma_variant_name(int cls, int v) {
    static const char *names[kMfmaClasses][8] = {
        {"lu_mfma_f32<2,1,2>", "lu_mfma_f32<2,1,1>", "lu_mfma_f32<2,2,2>"},
        {"lu_mfma_f32<4,1,2,4>", "lu_mfma_f32<4,1,2,3>", "lu_mfma_f32<4,2,2,5>", "lu_mfma_f32<4,2,2,4>",
         "lu_mfma_f32<4,2,2>", "lu_mfma_f32<4,1,2>", "lu_mfma_f32<4,1,1>", "lu_mfma_f32<4,1,1,3>"},
        {"lu_mfma_f32<6,2,2,3>", "lu_mfma_f32<6,2,4>", "lu_mfma_f32<6,2,2>", "lu_mfma_f32<6,3,2>",
         "lu_mfma_f32<6,2,2,4>"},
        {"lu_mfma_f32<8,2,4>"},
        {"lu_mfma_f32<9,3,4>"},
        {"lu_mfma_f32<12,2,4>"}};
    return (cls >= 0 && cls < kMfmaClasses && v >= 0 && v < mfma_variants(cls)) ? names[cls][v] : "";
}

hipError_t launch_lu_mfma(int cls, int v, const LuLaunch &a, hipStream_t st) {
    if (!a.list && a.nitems <= 0) return hipSuccess;
    switch (cls * 8 + v) {
        case 0: return launch_mfma<2, 1, 2>(a, st);
        case 1: return launch_mfma<2, 1, 1>(a, st);
        case 2: return launch_mfma<2, 2, 2>(a, st);
        case 8: return launch_mfma<4, 1, 2, 4>(a, st);
        case 9: return launch_mfma<4, 1, 2, 3>(a, st);
        case 10: return launch_mfma<4, 2, 2, 5>(a, st);
        case 11: return launch_mfma<4, 2, 2, 4>(a, st);
        case 12: return launch_mfma<4, 2, 2>(a, st);
        case 13: return launch_mfma<4, 1, 2>(a, st);
        case 14: return launch_mfma<4, 1, 1>(a, st);
        case 15: return launch_mfma<4, 1, 1, 3>(a, st);
        case 16: return launch_mfma<6, 2, 2, 3>(a, st);
        case 17: return launch_mfma<6, 2, 4>(a, st);
        case 18: return launch_mfma<6, 2, 2>(a, st);
        case 19: return launch_mfma<6, 3, 2>(a, st);
        case 20: return launch_mfma<6, 2, 2, 4>(a, st);
        case 24: return launch_mfma<8, 2, 4>(a, st);
        case 32: return launch_mfma<9, 3, 4>(a, st);
        case 40: return launch_mfma<12, 2, 4>(a, st);
        default: return hipErrorInvalidValue;
    }
}

size_t lu_big_lds_bytes(int ldw) {
    return sizeof(double2) * ((size_t)ldw * kPanel + kPanel * 64 + 2 * (size_t)ldw);
}

hipError_t launch_lu_big(const LuLaunch &a, double2 *work, int ldw, int nwg, hipStream_t st) {
    if (!a.list && a.nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(lu_big_f64, dim3(nwg), dim3(kBigThreads), lu_big_lds_bytes(ldw), st, a.job_block,
                       a.job_prefix, a.njobs, a.nitems, a.list, a.list_count, a.blocks, a.insts,
                       (const double2 *)a.pool, a.rbpool, a.eigpool, work, ldw, a.contrib, a.status);
    return hipGetLastError();
}

size_t pair_schur_lds_bytes(int ldw) {
    return sizeof(double2) * ((size_t)ldw * kPanel + kPanel * 64 + (size_t)ldw) + sizeof(int) * (size_t)ldw;
}

hipError_t launch_pair_schur(const PairDev *jobs, const int64_t *prefix, int njobs, int64_t npairs, int nwg,
                             double2 *pool, const int32_t *permpool, const double *eigpool, double2 *work, int ldw,
                             double2 *eigc, int *status, hipStream_t st) {
    if (npairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(pair_schur_f64, dim3(nwg), dim3(kBigThreads), pair_schur_lds_bytes(ldw), st, jobs, prefix,
                       njobs, npairs, pool, permpool, eigpool, work, ldw, eigc, status);
    return hipGetLastError();
}

hipError_t launch_schur_build(const SchurDev *jobs, const int64_t *prefix, int njobs, int64_t nwg, int maxA,
                              const double2 *pool_in, const double *eigpool, double2 *pool_out, float2 *pool32_out,
                              hipStream_t st) {
    if (nwg <= 0) return hipSuccess;
    const size_t lds = sizeof(double2) * (size_t)maxA * (1 + kSchurRows);
    hipLaunchKernelGGL(schur_build_f64, dim3((unsigned)nwg), dim3(256), lds, st, jobs, prefix, njobs, pool_in,
                       eigpool, pool_out, pool32_out);
    return hipGetLastError();
}

int schur_rows_per_wg() { return kSchurRows; }

hipError_t launch_combine(const InstDev *insts, const int64_t *inst_pt_prefix, int n_inst, int64_t npts,
                          const double2 *contrib, double2 *logg, double2 *gval, hipStream_t st) {
    if (npts <= 0) return hipSuccess;
    hipLaunchKernelGGL(combine_points, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, st, insts,
                       inst_pt_prefix, n_inst, npts, contrib, logg, gval);
    return hipGetLastError();
}

hipError_t launch_density_expand(const InstDev *insts, const int32_t *dinst, const int64_t *dprefix, int nd,
                                 int64_t npts, int64_t lds_values, const BlockDev *blocks, const int32_t *rbpool,
                                 const double2 *contrib, const double2 *tpool, double2 *logg, double2 *table,
                                 hipStream_t st) {
    if (npts <= 0) return hipSuccess;
    if (lds_values < 0 || lds_values > kDensityLdsValues) return hipErrorInvalidValue;
    hipLaunchKernelGGL(density_expand, dim3((unsigned)npts), dim3(256), sizeof(double2) * (size_t)lds_values, st,
                       insts, dinst, dprefix, nd, lds_values, blocks, rbpool, contrib, tpool, logg, table);
    return hipGetLastError();
}

hipError_t launch_density_hermitize(const InstDev *insts, const int32_t *dinst, const int64_t *mprefix, int nd,
                                    int64_t nmat, int64_t lds_values, const double2 *bufA, const double2 *bufB,
                                    double *out, hipStream_t st) {
    if (nmat <= 0) return hipSuccess;
    if (lds_values < 0 || lds_values > kDensityLdsValues) return hipErrorInvalidValue;
    hipLaunchKernelGGL(density_hermitize, dim3((unsigned)nmat), dim3(256), sizeof(double2) * (size_t)lds_values, st,
                       insts, dinst, mprefix, nd, lds_values, bufA, bufB, out);
    return hipGetLastError();
}

hipError_t launch_dft_cols(const DftStageDev *st_dev, const int64_t *prefix, int n, int64_t total, const double2 *tw,
                           const double2 *in, double2 *out, double *probs, double *err, const int *status,
                           hipStream_t st) {
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(dft_cols<kDftColsK>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, st_dev, prefix,
                       n, total, tw, in, out, probs, err, status);
    return hipGetLastError();
}

hipError_t launch_dft_stage(const DftStageDev *st_dev, const int64_t *prefix, int n, int64_t total, const double2 *tw,
                            const double2 *in, double2 *out, double *probs, double *err, const int *status,
                            hipStream_t st) {
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(dft_stage, dim3((unsigned)((4 * total + 255) / 256)), dim3(256), 0, st, st_dev, prefix, n,
                       total, tw, in, out, probs, err, status);
    return hipGetLastError();
}


}  // namespace cgd

namespace cgd {
hipError_t launch_zero_ints(int *p, int n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_ints, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long *p, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_u64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_mixed_cut(const InstDev *insts, const int64_t *inst_pt_prefix, int n_inst, int64_t npts,
                            const double2 *logg, double tol, unsigned long long *hist, int *cut, hipStream_t st) {
    if (n_inst <= 0) return hipSuccess;
    hipError_t e = launch_zero_u64(hist, (int64_t)n_inst * kMixedBuckets, st);
    if (e != hipSuccess) return e;
    if (npts > 0) {
        hipLaunchKernelGGL(mixed_hist, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, st, insts,
                           inst_pt_prefix, n_inst, npts, logg, hist);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(mixed_cut, dim3(n_inst), dim3(64), 0, st, insts, n_inst, tol, hist, cut);
    return hipGetLastError();
}

hipError_t launch_select_points(const InstDev *insts, const int64_t *inst_pt_prefix, int n_inst, int64_t npts,
                                const BlockDev *blocks, const double2 *logg, const int *cut, int2 *list_base,
                                const int64_t *list_off, int *counts, int n_lists, hipStream_t st) {
    if (npts <= 0) return hipSuccess;
    hipLaunchKernelGGL(select_points, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, st, insts,
                       inst_pt_prefix, n_inst, npts, blocks, logg, cut, list_base, list_off, counts, n_lists);
    return hipGetLastError();
}

hipError_t launch_mixed_err(const InstDev *insts, int n_inst, const double2 *logg, const int *cut, double *err,
                            const int *status, hipStream_t st) {
    if (n_inst <= 0 || !err) return hipSuccess;
    hipLaunchKernelGGL(mixed_err, dim3(n_inst), dim3(256), 0, st, insts, logg, cut, err, status);
    return hipGetLastError();
}
}  // namespace cgd

namespace cgd {
template <int PR, int PC, int TR, int TC>
static hipError_t launch_adj(const AdjArgs &a, int nitems, hipStream_t st) {
    hipLaunchKernelGGL((lu_adjoint<PR, PC, TR, TC>), dim3(nitems), dim3(PR * PC), 0, st, a);
    return hipGetLastError();
}

int adj_class_limit(int cls) {
    switch (cls) {
        case 0: return 32;
        case 1: return 64;
        case 2: return 96;
        case 3: return kAdjBigMax;
        default: return 0;
    }
}

hipError_t prepare_adj_big(int ldw) {
    return hipFuncSetAttribute((const void *)adj_big_f64, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)adj_big_lds_bytes(ldw));
}

hipError_t launch_adjoint(int cls, const AdjArgs &a0, int nitems, int64_t item_base, hipStream_t st) {
    if (nitems <= 0) return hipSuccess;
    AdjArgs a = a0;
    a.item_base = (int)item_base;
    switch (cls) {
        case 0: return launch_adj<8, 8, 4, 4>(a, nitems, st);
        case 1: return launch_adj<16, 16, 4, 4>(a, nitems, st);
        case 2: return launch_adj<16, 32, 6, 3>(a, nitems, st);
        case 3: {
            if (a.work == nullptr || a.ldw <= 0 || a.nwg <= 0) return hipErrorInvalidValue;
            const int grid = nitems < a.nwg ? nitems : a.nwg;
            hipLaunchKernelGGL(adj_big_f64, dim3(grid), dim3(kBigThreads), adj_big_lds_bytes(a.ldw), st, a, nitems);
            return hipGetLastError();
        }
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_adjoint_reduce(const GradBlockDev *gblocks, const int64_t *elem_prefix, int ngb, int64_t total,
                                 const double2 *partial, int64_t part_stride, double2 *zout, hipStream_t st) {
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(adjoint_reduce, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, gblocks,
                       elem_prefix, ngb, total, partial, part_stride, zout);
    return hipGetLastError();
}

hipError_t launch_adjoint_gather(const InstDev *insts, const int64_t *inst_pt_prefix, int n_inst, int64_t npts,
                                 const int64_t *buf_off, const double2 *bufA, const double2 *bufB, double2 *ghat,
                                 hipStream_t st) {
    if (npts <= 0) return hipSuccess;
    hipLaunchKernelGGL(adjoint_gather, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, st, insts, inst_pt_prefix,
                       n_inst, npts, buf_off, bufA, bufB, ghat);
    return hipGetLastError();
}

hipError_t launch_adjoint_seed(const InstDev *insts, const int64_t *prob_prefix, int n_inst, int64_t nprobs,
                               const double *dprobs, const int64_t *buf_off, double2 *out, hipStream_t st) {
    if (nprobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(adjoint_seed, dim3((unsigned)((nprobs + 255) / 256)), dim3(256), 0, st, insts, prob_prefix,
                       n_inst, nprobs, dprobs, buf_off, out);
    return hipGetLastError();
}
}  // namespace cgd

namespace cgd {
// Dynamic LDS limits of the kernels that need more than the default; called
// once at context creation (not inside a captured launch sequence).
int hess_class_limit(int cls) {
    switch (cls) {
        case 0: return 32;
        case 1: return 64;
        case 2: return 96;
        case 3: return 144;
        default: return 0;
    }
}

template <int TY, int TX, int R, int SC>
static hipError_t launch_hr(const HessDev *jobs, const int64_t *prefix, int njobs, int64_t nwg, double2 *pool,
                            const double *eigpool, double2 *eigc, hipStream_t st) {
    hipLaunchKernelGGL((hess_reduce_f64<TY, TX, R, SC>), dim3((unsigned)nwg), dim3(TX * TY), sizeof(HessLds<TY, TX, R, SC>),
                       st, jobs, prefix, njobs, pool, eigpool, eigc);
    return hipGetLastError();
}

hipError_t launch_hess_reduce(int cls, const HessDev *jobs, const int64_t *prefix, int njobs, int64_t nwg,
                              double2 *pool, const double *eigpool, double2 *eigc, hipStream_t st) {
    if (nwg <= 0) return hipSuccess;
    switch (cls) {
        case 0: return launch_hr<16, 32, 2, 1>(jobs, prefix, njobs, nwg, pool, eigpool, eigc, st);
        case 1: return launch_hr<16, 32, 4, 2>(jobs, prefix, njobs, nwg, pool, eigpool, eigc, st);
        case 2: return launch_hr<16, 32, 6, 3>(jobs, prefix, njobs, nwg, pool, eigpool, eigc, st);
        case 3: return launch_hr<32, 16, 5, 9>(jobs, prefix, njobs, nwg, pool, eigpool, eigc, st);
        default: return hipErrorInvalidValue;
    }
}

static constexpr int hess_det_lds_bytes(int MB) { return 2 * 16 * 16 * MB * (int)sizeof(double2); }

template <int MB>
static hipError_t launch_hd(const HessDev *jobs, const int64_t *prefix, int njobs, int64_t nwg, const double2 *pool,
                            const double2 *eigc, double2 *table, int *status, hipStream_t st) {
    hipLaunchKernelGGL((hess_det_f64<MB>), dim3((unsigned)nwg), dim3(kHessDetThreads), hess_det_lds_bytes(MB), st,
                       jobs, prefix, njobs, pool, eigc, table, status);
    return hipGetLastError();
}

hipError_t launch_hess_det(int cls, const HessDev *jobs, const int64_t *prefix, int njobs, int64_t nwg,
                           const double2 *pool, const double2 *eigc, double2 *table, int *status, hipStream_t st) {
    if (nwg <= 0) return hipSuccess;
    switch (cls) {
        case 0: return launch_hd<2>(jobs, prefix, njobs, nwg, pool, eigc, table, status, st);
        case 1: return launch_hd<4>(jobs, prefix, njobs, nwg, pool, eigc, table, status, st);
        case 2: return launch_hd<6>(jobs, prefix, njobs, nwg, pool, eigc, table, status, st);
        case 3: return launch_hd<9>(jobs, prefix, njobs, nwg, pool, eigc, table, status, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_hess_scatter(const HessDev *jobs, const int64_t *prefix, int njobs, int64_t total,
                               const InstDev *insts, const double2 *table, double2 *contrib, hipStream_t st) {
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(hess_scatter, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, jobs, prefix, njobs,
                       total, insts, table, contrib);
    return hipGetLastError();
}

hipError_t prepare_kernels(int big_ldw, int schur_maxA, int pair_ldw) {
    for (hipError_t e : {hipFuncSetAttribute((const void *)hess_reduce_f64<16, 32, 2, 1>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(HessLds<16, 32, 2, 1>)),
                         hipFuncSetAttribute((const void *)hess_reduce_f64<16, 32, 4, 2>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(HessLds<16, 32, 4, 2>)),
                         hipFuncSetAttribute((const void *)hess_reduce_f64<16, 32, 6, 3>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(HessLds<16, 32, 6, 3>)),
                         hipFuncSetAttribute((const void *)hess_reduce_f64<32, 16, 5, 9>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(HessLds<32, 16, 5, 9>)),
                         hipFuncSetAttribute((const void *)hess_det_f64<9>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                             hess_det_lds_bytes(9)),
                         hipFuncSetAttribute((const void *)density_expand, hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)(sizeof(double2) * kDensityLdsValues)),
                         hipFuncSetAttribute((const void *)density_hermitize, hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)(sizeof(double2) * kDensityLdsValues))})
        if (e != hipSuccess) return e;
    for (hipError_t e : {prepare_mfma<2, 1, 2>(), prepare_mfma<2, 1, 1>(), prepare_mfma<2, 2, 2>(),
                         prepare_mfma<4, 2, 2>(), prepare_mfma<4, 1, 2>(), prepare_mfma<4, 1, 1>(),
                         prepare_mfma<4, 1, 1, 3>(), prepare_mfma<6, 2, 4>(), prepare_mfma<6, 2, 2>(),
                         prepare_mfma<6, 3, 2>(), prepare_mfma<8, 2, 4>(), prepare_mfma<9, 3, 4>(),
                         prepare_mfma<12, 2, 4>(), prepare_mfma<4, 2, 2, 4>(), prepare_mfma<4, 1, 2, 3>(),
                         prepare_mfma<6, 2, 2, 3>(), prepare_mfma<4, 2, 2, 5>(), prepare_mfma<4, 1, 2, 4>(),
                         prepare_mfma<6, 2, 2, 4>(), prepare_mfma64<2, 1, 1>(), prepare_mfma64<2, 1, 2>(),
                         prepare_mfma64<2, 1, 1, 3>(), prepare_mfma64<4, 2, 2>(), prepare_mfma64<4, 1, 2>(),
                         prepare_mfma64<4, 2, 2, 3>(), prepare_mfma64<6, 2, 2>(), prepare_mfma64<6, 2, 4>(),
                         prepare_mfma64<6, 3, 2>()})
        if (e != hipSuccess) return e;
    if (big_ldw > 0) {
        const hipError_t e = hipFuncSetAttribute((const void *)lu_big_f64, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)lu_big_lds_bytes(big_ldw));
        if (e != hipSuccess) return e;
    }
    if (pair_ldw > 0) {
        const hipError_t e = hipFuncSetAttribute((const void *)pair_schur_f64,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)pair_schur_lds_bytes(pair_ldw));
        if (e != hipSuccess) return e;
    }
    if (schur_maxA > 0) {
        const hipError_t e = hipFuncSetAttribute((const void *)schur_build_f64,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)(sizeof(double2) * (size_t)schur_maxA * (1 + kSchurRows)));
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
}  // namespace cgd

// ---------------------------------------------------------------------------
// Static per-device scratch for cgd_eval_static, the evaluation entry point
// that allocates nothing.  `scratch` is a host-side stand-in in host code; its
// device address on each GPU comes from hipGetSymbolAddress, taken once per
// device (with that device current) and kept in g_scratch.  Every call on a
// GPU shares that GPU's array.
// ---------------------------------------------------------------------------
#include <mutex>

namespace cgd {

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch_setup(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[dev]) return hipSuccess;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch[dev] = ptr;
    return hipSuccess;
}

void *static_scratch(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch[dev];
}

}  // namespace cgd
