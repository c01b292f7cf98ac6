// Internal descriptors shared by the host side of the C ABI and the HIP kernels.
#pragma once
#include <stdint.h>
#include <stddef.h>

#include <hip/hip_runtime.h>

namespace cgd {

constexpr int kMaxBins = 8;

// One instance on the device.  The evaluated grid is the half grid
// k_1 in [0, G_1/2], k_2..k_L in [0, G_l) (row-major, k_L fastest); the other
// half follows from G(conj w) = conj G(w) because the coefficients are real.
struct InstDev {
    int32_t L;
    int32_t nblocks;          // internal-mode blocks contributing to each point
    int32_t G[kMaxBins];      // grid extents
    int32_t N[kMaxBins];      // cutoffs
    int32_t H1;               // G_1/2 + 1
    int32_t pad;
    int64_t npts;             // evaluated points = H1 * prod_{l>=2} G_l
    int64_t pt_off;           // first evaluated point of this instance (global point index)
    int64_t c_off;            // first contribution slot: c_off + p * nblocks + blk
    int64_t prob_off;         // first output probability
    int64_t nprobs;           // prod (N_l + 1)
    double logpr0_re, logpr0_im;  // constant part of log G (vacuum probability, traced modes)
    int32_t first_block;      // this instance's blocks are first_block .. first_block + nblocks - 1
    int32_t pad2;
    double rho;               // 0: grid on the unit circle, w = exp(2 pi i k / G); > 0 (moments mode):
                              // w = exp(t), t = rho exp(2 pi i k / G) on a circle of radius rho
    double tau;               // mixed path: relative error bound assumed for an FP32 value of G (0: no FP32 block)
    int32_t dft_log;          // 1: the DFT takes log G instead of G (cumulants)
    int32_t nvar;             // density mode: 2 g generating-function variables of the g kept modes (0: off)
    int32_t fock_n;           // density mode: Fock cutoff N of every kept mode
    int32_t pad5;
    int64_t E;                // values per evaluated point: (N + 1)^(2 g) in density mode, else 1
    int64_t gv_off;           // first value of this instance in the per-point value table (and DFT buffers)
    int32_t tw_off[kMaxBins]; // axis l: first of its G_l twiddles exp(-2 pi i m / G_l) in the twiddle table
};

// One factorisation job family: an (instance, internal block) pair.  Every
// evaluated point of the instance factorises S = I - diag(d(w)) Hs, where Hs
// is either the block's (reduced, possibly bordered) matrix H (hs_stride = 0)
// or, after eliminating the first bin through its eigenbasis, the per-k_1
// Schur matrix C(w_1) stored at h_off + k_1 * hs_stride.
struct BlockDev {
    int32_t inst;
    int32_t blk;
    int32_t nb;               // matrix order including the border row/column
    int32_t bordered;         // 1: last row/column is the displacement border
    int32_t schur_axis;       // bin eliminated through its eigenbasis (-1: none)
    int32_t n_eig;            // number of eliminated eigen-directions
    int64_t h_off;            // complex offset of the matrix (row-major, ld = nb)
    int64_t hs_stride;        // complex stride per k of the eliminated bin (0: one matrix)
    int64_t rb_off;           // offset of nb row-bin indices (-1: factor 1)
    int64_t eig_off;          // offset of the eliminated bin's eigenvalues
    int32_t cls;              // FP64 size class: register classes 0..kRegClasses-1, kRegClasses = blocked
    int32_t fp32;             // mixed path: 1 if the first pass factorises this block in FP32
    int32_t nkeep;            // density mode: rows of the kept-mode border (2 g_k), before the gamma border
    int32_t pad;
    int64_t t_off;            // density mode: trailing Schur complement (nkeep + bordered)^2 per point
    int64_t kv_off;           // density mode: nkeep generating-function variable indices (in rbpool)
    int32_t lowrank;          // > 0: low-rank block of that rank (no factorisation; lowrank_points)
    int32_t pad2;
    int64_t lr_off;           // its (L + 1) r x r matrices G_t, G_0 .. G_{L-1} in the pool
};

constexpr int kLowRankMax = 4;  // largest rank taken by the low-rank route (two squeezed inputs)

// Build of the Schur matrices C(w_A) = H_BB + P diag(w_A / (1 - w_A lambda)) Q
// for every value k of the eliminated bin A (P = H_BA V, Q = V^H H_AB with
// H_AA = V diag(lambda) V^H).
struct SchurDev {
    int32_t inst;
    int32_t axis;             // eliminated bin
    int32_t nA, nB;
    int32_t nk;               // number of k values (H1 for axis 0, else G_axis)
    int32_t Gax;              // grid extent of the eliminated axis
    int64_t p_off, q_off, hbb_off, eig_off, c_off;
    double rho;               // circle radius of the instance (see InstDev)
};

// Hessenberg route: a block whose rows left after eliminating bin A (axis
// axA) all lie in one bin (axis axB).  For each value k_A the Schur matrix
// C(w_A) at c_off + k_A n^2 is reduced to Hessenberg form in place; every
// pair (k_A, k_B) then costs one O(n^2) factorisation, stored at
// t_off + k_A dB + k_B and copied to the points.
struct HessDev {
    int32_t inst, blk, n;
    int32_t axA, axB;
    int32_t dA, dB;           // number of k_A and k_B values (half grid on axis 0)
    int32_t GB;               // grid extent of axis B
    int32_t n_eig;
    int32_t cls;              // size class (n <= 32, 64, 96, 144)
    int32_t GA;               // grid extent of axis A
    int32_t axP, dP;          // pair route: the middle axis and its number of values (axP = -1: none);
                              // the matrix index kA then runs over (k_A, k_P) pairs, kA_axis * dP + k_P
    int64_t c_off, eig_off, t_off, ec_off;
    double rho;               // circle radius of the instance (see InstDev)
};

// Pair route: a block whose rows left after the eigenbasis elimination of
// axis A lie in two bins, P and B.  For every (w_A, w_P) pair the rows of P
// are eliminated by a partial LU of F = [[I - w_P C_PP, -w_P C_PB], [C_BP, C_BB]]
// (C = C(w_A), bin-P rows first), which leaves S = C_BB + w_P C_BP
// (I - w_P C_PP)^-1 C_PB, so that det(I - D C) = det(I - w_P C_PP) det(I - w_B S).
struct PairDev {
    int32_t inst, n, nP;      // order, rows of bin P (the pivots taken)
    int32_t axA, axP;         // eliminated axis, partial-LU axis
    int32_t dA, dP;           // number of values of k_A and k_P
    int32_t GA, GP;           // their grid extents
    int32_t n_eig;            // eigenvalues of the eliminated bin
    int64_t c_off, hs_stride; // C(w_A) in the matrix pool, stride per value of k_A
    int64_t perm_off;         // row order of F (int32 pool): bin P rows, then bin B rows
    int64_t eig_off;
    int64_t s_off;            // S, (n - nP)^2 per pair, in the matrix pool
    int64_t ec_off;           // per pair: sum Log(1 - w_A lambda_i) + log det(I - w_P C_PP)
    double rho;               // circle radius of the instance (see InstDev)
};

// Gradient: one internal block with its full (bordered) matrix, no reduction.
struct GradBlockDev {
    int32_t inst;
    int32_t nb;               // order including the border
    int32_t bordered;
    int32_t nchunks;          // chunks of grid points (work items) of this block
    int64_t h_off;            // complex offset of the bordered H in the gradient pool
    int64_t rb_off;           // row bins (nb entries)
    int64_t first_item;       // first adjoint work item
    int64_t z_off;            // output: n*n (Z_H) + n (Z_gamma) + 1 (Z_0), n = nb - bordered
};

struct AdjArgs {
    const int32_t *job_block;  // gradient block per job
    const int64_t *job_prefix; // first item of each job
    int njobs;
    int chunk;                 // grid points per item
    const GradBlockDev *gblocks;
    const InstDev *insts;
    const double2 *pool;
    const int32_t *rbpool;
    const double2 *logg;
    const double2 *ghat;
    double2 *partial;
    int64_t part_stride;
    int item_base;             // absolute index of the launch's first item
    double2 *work;             // orders above the register classes: ldw x ldw workspace per workgroup
    int ldw;
    int nwg;                   // workgroups (each loops over items)
};

// One axis pass of the separable inverse DFT for one instance.
struct DftStageDev {
    int32_t inst, K, Bout, G;
    int32_t final_stage, moments;  // moments: scale output index b by b! / rho^b (Taylor coefficient -> derivative)
    int32_t density, pad;          // density mode: complex output to `out`, half-grid weights already applied
    int64_t outer, inner, in_off, out_off;
    int64_t tw_off;           // exp(-2 pi i m / G), m = 0 .. G-1, in the twiddle pool
    double scale;
    double rho;
};

struct LuLaunch {
    const int32_t *job_block;
    const int64_t *job_prefix;
    int njobs;
    int64_t nitems;
    const int2 *list;          // explicit (block, point) items, or nullptr
    const int *list_count;
    int64_t list_capacity;
    const BlockDev *blocks;
    const InstDev *insts;
    const void *pool;          // double2 or float2 matrices
    const int32_t *rbpool;
    const double *eigpool;
    double2 *contrib;
    int *status;
    double2 *tpool;            // density mode: trailing Schur complements
    const double2 *tw;         // twiddles exp(-2 pi i m / G) (InstDev::tw_off), or nullptr
    const int32_t *job_hint;   // per 64 items: the job of the chunk's first item (range launches), or nullptr
};

// launchers (cgd_kernels.hip)
int reg_class_limit(int cls);          // max matrix order of register class cls (0 = none)
constexpr int kRegClasses = 5;
// shape variants per class: reg_variants(cls) thread grids of the FP64
// register kernel, mfma_variants(cls) wave layouts of the FP32 MFMA kernel
// (variant 0 is the default; the autotuner of cgd_create picks one)
int reg_variants(int cls);
int reg_kernel_variants(int cls);      // the first ones: register-kernel shapes (density mode needs one)
const char *reg_variant_name(int cls, int v);
hipError_t launch_lu_reg(int cls, int v, const LuLaunch &a, hipStream_t st);
// low-rank blocks of rank r (1..kLowRankMax): per (block, point) the r x r determinant
// det(I - G_t - sum_l w_l G_l); job j covers blocks lrblk[jobs[j].x .. + jobs[j].y) of
// one instance, in tiles of 16 blocks x lowrank_points_per_tile() points (prefix: tiles
// before job j; ntiles in all); gstride >= (L + 1) r^2 and wstride >= L over every job
hipError_t launch_lowrank_points(int r, const int2 *jobs, const int64_t *prefix, int njobs, int64_t ntiles,
                                 const int32_t *lrblk, const BlockDev *blocks, const InstDev *insts,
                                 const double2 *pool, const double2 *tw, double2 *contrib, int *status,
                                 int gstride, int wstride, hipStream_t st);
int lowrank_points_per_tile();
// FP64 factorisations of order <= 16 (range launches): lu_mfma_f64<1,1,1>
hipError_t launch_lu_one_tile(const LuLaunch &a, hipStream_t st);
constexpr int kMfmaClasses = 6;
int mfma_class_limit(int cls);         // max matrix order of FP32 MFMA class cls
int mfma_variants(int cls);
const char *mfma_variant_name(int cls, int v);
hipError_t launch_lu_mfma(int cls, int v, const LuLaunch &a, hipStream_t st);
size_t lu_big_lds_bytes(int ldw);
hipError_t prepare_kernels(int big_ldw, int schur_maxA, int pair_ldw);
hipError_t launch_lu_big(const LuLaunch &a, double2 *work, int ldw, int nwg, hipStream_t st);
hipError_t launch_schur_build(const SchurDev *jobs, const int64_t *prefix, int njobs, int64_t nwg, int maxA,
                              const double2 *pool_in, const double *eigpool, double2 *pool_out, float2 *pool32_out,
                              hipStream_t st);
// adjoint
int adj_class_limit(int cls);
constexpr int kAdjClasses = 4;  // 0..2: register kernels (orders <= 96); 3: blocked, workspace in HBM
constexpr int kAdjBigMax = 481;  // largest bordered order of class 3 (its LDS: 151 KB)
size_t adj_big_lds_bytes(int ldw);
hipError_t prepare_adj_big(int ldw);
hipError_t launch_adjoint(int cls, const AdjArgs &a, int nitems, int64_t item_base, hipStream_t st);
hipError_t launch_adjoint_reduce(const GradBlockDev *gblocks, const int64_t *elem_prefix, int ngb, int64_t total,
                                 const double2 *partial, int64_t part_stride, double2 *zout, hipStream_t st);
hipError_t launch_adjoint_gather(const InstDev *insts, const int64_t *inst_pt_prefix, int n_inst, int64_t npts,
                                 const int64_t *buf_off, const double2 *bufA, const double2 *bufB, double2 *ghat,
                                 hipStream_t st);
hipError_t launch_adjoint_seed(const InstDev *insts, const int64_t *prob_prefix, int n_inst, int64_t nprobs,
                               const double *dprobs, const int64_t *buf_off, double2 *out, hipStream_t st);
// mixed path
hipError_t launch_zero_ints(int *p, int n, hipStream_t st);
// buckets of |G| per instance for the FP32/FP64 split of the mixed path
constexpr int kMixedBucketsPerOctave = 4;
constexpr int kMixedBuckets = 64 * kMixedBucketsPerOctave;
hipError_t launch_zero_u64(unsigned long long *p, int64_t n, hipStream_t st);
hipError_t launch_mixed_cut(const InstDev *insts, const int64_t *inst_pt_prefix, int n_inst, int64_t npts,
                            const double2 *logg, double tol, unsigned long long *hist, int *cut, hipStream_t st);
hipError_t launch_select_points(const InstDev *insts, const int64_t *inst_pt_prefix, int n_inst, int64_t npts,
                                const BlockDev *blocks, const double2 *logg, const int *cut, int2 *list_base,
                                const int64_t *list_off, int *counts, int n_lists, hipStream_t st);
hipError_t launch_mixed_err(const InstDev *insts, int n_inst, const double2 *logg, const int *cut, double *err,
                            const int *status, hipStream_t st);
// Hessenberg route
constexpr int kHessClasses = 4;
int hess_class_limit(int cls);          // max order of class cls: 32, 64, 96, 144
hipError_t launch_hess_reduce(int cls, const HessDev *jobs, const int64_t *prefix, int njobs, int64_t nwg,
                              double2 *pool, const double *eigpool, double2 *eigc, hipStream_t st);
hipError_t launch_hess_det(int cls, const HessDev *jobs, const int64_t *prefix, int njobs, int64_t nwg,
                           const double2 *pool, const double2 *eigc, double2 *table, int *status, hipStream_t st);
hipError_t launch_pair_schur(const PairDev *jobs, const int64_t *prefix, int njobs, int64_t npairs, int nwg,
                             double2 *pool, const int32_t *permpool, const double *eigpool, double2 *work, int ldw,
                             double2 *eigc, int *status, hipStream_t st);
size_t pair_schur_lds_bytes(int ldw);
hipError_t launch_hess_scatter(const HessDev *jobs, const int64_t *prefix, int njobs, int64_t total,
                               const InstDev *insts, const double2 *table, double2 *contrib, hipStream_t st);
int schur_rows_per_wg();
hipError_t launch_combine(const InstDev *insts, const int64_t *inst_pt_prefix, int n_inst, int64_t npts,
                          const double2 *contrib, double2 *logg, double2 *gval, hipStream_t st);
// density mode: per point, the kept modes' generating function from the
// trailing Schur complements, expanded into the (N+1)^(2g) matrix elements
constexpr int kMaxKeepVars = 16;
constexpr int64_t kDensityLdsValues = 4096;
hipError_t launch_density_expand(const InstDev *insts, const int32_t *dinst, const int64_t *dprefix, int nd,
                                 int64_t npts, int64_t lds_values, const BlockDev *blocks, const int32_t *rbpool,
                                 const double2 *contrib, const double2 *tpool, double2 *logg, double2 *table,
                                 hipStream_t st);
hipError_t launch_density_hermitize(const InstDev *insts, const int32_t *dinst, const int64_t *mprefix, int nd,
                                    int64_t nmat, int64_t lds_values, const double2 *bufA, const double2 *bufB,
                                    double *out, hipStream_t st);
// axis passes with extent K <= kDftColsK: one thread per column (dft_cols)
constexpr int kDftColsK = 16;
hipError_t launch_dft_cols(const DftStageDev *st_dev, const int64_t *prefix, int n, int64_t total, const double2 *tw,
                           const double2 *in, double2 *out, double *probs, double *err, const int *status,
                           hipStream_t st);
hipError_t launch_dft_stage(const DftStageDev *st_dev, const int64_t *prefix, int n, int64_t total, const double2 *tw,
                            const double2 *in, double2 *out, double *probs, double *err, const int *status,
                            hipStream_t st);

// static per-device scratch of cgd_eval_static (cgd_kernels.hip)
constexpr size_t kStaticScratchBytes = (size_t)128 << 20;
hipError_t static_scratch_setup(int dev);  // with device dev current; once per device
void *static_scratch(int dev);             // its device address, or nullptr before setup

}  // namespace cgd
