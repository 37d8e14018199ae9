// Internal declarations shared by the library's translation units.
//
// Data layout in device memory (one handle = `B` members of one shape):
//   field block   [t][j][node]        n_t * n_xi * (n+1)^2 values, zero boundary ring
//   KKT vector    [y | u | lambda]    three field blocks
//   batch         [member][...]       members back to back
// A "column" is one (member, t, j) slice of (n+1)^2 nodes; kernels address
// columns through ColMap so that the same kernel serves a KKT vector, a
// scratch block, a degree level of the hierarchical sweep or a multigrid level.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/sg.h"

namespace sg {

struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define SG_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            throw ::sg::Error(SG_ERR_HIP, std::string(#call) + " failed: " + hipGetErrorString(e_)); \
    } while (0)

constexpr int kMaxM = 16;        // random variables
constexpr int kMaxP = 8;         // polynomial degree
constexpr int kMaxLevels = 12;   // multigrid levels (n <= 4096 down to 8)
constexpr int kMaxSmooth = 4;    // Chebyshev smoothing degree per side
constexpr int kCoarseN = 8;      // coarsest multigrid grid (elements per side)
constexpr int kCoarsePad = 64;   // (kCoarseN-1)^2 = 49 unknowns padded for MFMA tiles
constexpr int kMaxRestart = 64;
constexpr int kPinnedDoubles = 16384;   // host-pinned scratch per handle (readbacks and uploads, up to 2048 members)

// Per-member scalars used by the kernels (device array, one entry per member).
struct MemberDev {
    double beta, gamma, tau;   // tau = 1 for steady problems
    double c0;                 // constant mean coefficient kappa_0
    double a1, b1;             // mean block A1 = a1 K_unit + b1 M
    double off_scale;          // factor on off-level products (1 steady, tau time)
    double hg;                 // 1 + gamma
};

// Per-member, per-multigrid-level constants (device array [member][level]).
struct LevelDev {
    double wc, we, wd;               // 9-point stencil weights of a1 K + b1 M_h: centre, edge, corner
    double dinv;                     // 1 / diagonal
    double pre[kMaxSmooth][2];       // Chebyshev smoothing steps (c_d, c_r), pre
    double post[kMaxSmooth][2];      // post
};

// Column addressing: column c in [0, ncols) -> member b = c / (L*nt),
// t = (c / L) % nt, local l = c % L, chaos j = j0 + l;
// address = base + b*mstride + t*tstride + j*nodes.
struct ColMap {
    int64_t mstride, tstride, nodes;
    int L, nt, j0;
    __host__ __device__ int64_t off(int c) const {
        int l = c % L;
        int q = c / L;
        int t = q % nt;
        int b = q / nt;
        return (int64_t)b * mstride + (int64_t)t * tstride + (int64_t)(j0 + l) * nodes;
    }
    __host__ __device__ int member(int c) const { return c / (L * nt); }
    __host__ __device__ int tstep(int c) const { return (c / L) % nt; }
    __host__ __device__ int chaos(int c) const { return j0 + c % L; }
};

inline ColMap contiguous_cols(int ncols, int64_t nodes) {
    ColMap m;
    m.mstride = 0; m.tstride = 0; m.nodes = nodes; m.L = ncols; m.nt = 1; m.j0 = 0;
    return m;
}

// Shape of a handle.
struct Shape {
    int n, M, P, nt;           // nt = 1 for steady
    bool time;
    int field = SG_FIELD_AFFINE;   // coefficient model of the batch
    int nA = 0;                    // coefficient terms: M + 1 (affine) or C(M + 2P, 2P) (log-normal)
    int nxi;
    int64_t nodes;             // (n+1)^2
    int64_t tstride;           // nxi * nodes
    int64_t blk;               // nt * nxi * nodes
    int off[kMaxP + 2];        // degree level offsets
    int nlev_mg;               // multigrid levels
    int mg_n[kMaxLevels];      // elements per side per multigrid level
    // node rows per strip of the sweep kernels, per element type [0 FP64, 1 FP32]
    // and kernel [SWEEP_APPLY, SWEEP_HGS, SWEEP_KKT]; chosen by the autotuner
    int sweep_rows[2][3] = {{4, 4, 4}, {4, 4, 4}};
};
enum SweepKind { SWEEP_APPLY = 0, SWEEP_HGS = 1, SWEEP_KKT = 2 };
constexpr int kSweepRowChoices[3] = {2, 4, 8};

// Host-side tables built by setup.
struct HostTables {
    std::vector<int32_t> alpha;       // [nxi][M]
    std::vector<int32_t> nbr_idx;     // [nxi][M][2]
    std::vector<double> nbr_val;      // [nxi][M][2]
};

// ---- kernel launchers (kernels.hip) ------------------------------------------
struct OpDev {                   // device pointers describing the operator of a handle
    const int32_t* nbr_idx;      // [nxi][M][2]
    const double* nbr_val;       // [nxi][M][2]
    const void* coef;            // [member][M+1][n][n] in T
    const double* coef64;        // the same in FP64 (the sweep kernels compute in FP64 for every storage type)
    int64_t coef_mstride;        // elements per member (0 = shared)
    const MemberDev* mem;        // [member]
    int mem_shared;              // 1 = all vectors use member 0
    const int* active;           // [vector] skip vectors whose flag is 0 (null: process all)
    // general chaos coupling (log-normal field): per-element B_e = sum_l kappa_l(e) H_l,
    // [member][e][i][j]; genBr keeps the terms l < truncation r (genB when r = n_A)
    const double* genB;
    const double* genBr;
    int64_t gen_mstride;         // elements per member (0 = shared)
    int gen;                     // 1: the general-coupling kernels
    double off_sign;             // hGS right-hand sides: base - off_sign * off_scale * (couplings); -1 adds them
};

// Element-sweep kernels (sweep.hip); return false when the shape needs the
// generic kernels (more than 8 random variables).
template <typename T>
bool launch_sgx_apply(const Shape& s, const OpDev& op, const T* x, T* y, int nvec, uint32_t mask, hipStream_t st);
template <typename T>
bool launch_sgx_kkt(const Shape& s, const OpDev& op, const T* x, T* y, int nvec, hipStream_t st);
template <typename T>
bool launch_sgx_hgs_rhs(const Shape& s, const OpDev& op, int d, uint32_t mask, int use_lower, int use_upper,
                        const T* base, ColMap bmap, const T* V, ColMap vmap, T* out, ColMap omap, int nmembers,
                        hipStream_t st);

// SG apply y = sum_k (G_k (x) K_k) x: the mean (k = 0) and the modes k with
// bit k-1 of `mask` set (all ones: the full operator; the truncated Z_r of
// Richardson steps keeps k < r).
template <typename T>
void launch_sg_apply(const Shape& s, const OpDev& op, const T* x, T* y, int nvec, uint32_t mask, hipStream_t st);

template <typename T>
void launch_kkt_apply(const Shape& s, const OpDev& op, const T* x, T* y, int nvec, hipStream_t st);

// hGS off-level right-hand side for degree level d:
//   out_j = base_j - off_scale * sum_{k in modes} K_k (g- V_{j-e_k} [lower] + g+ V_{j+e_k} [upper])
template <typename T>
void launch_hgs_rhs(const Shape& s, const OpDev& op, int d, uint32_t modes_mask, int use_lower,
                    int use_upper, const T* base, ColMap base_map, const T* V, ColMap v_map, T* out,
                    ColMap out_map, int nmembers, hipStream_t st);

// General chaos coupling (gen.hip): out_j = base_j + s sum_{i in [ilo1, ihi1) u
// [ilo2, ihi2)} sum_e (B_e[i][j] + [i == j] mean_c) (K_ref X_i|e) for the L
// output columns j0.. of every (vector, t) slice, B = genBr if trunc else genB,
// s = scale or (scale_off) -off_scale of the member; X field blocks of member
// stride xms and time stride xts.
template <typename T>
void launch_gen_sg(const Shape& s, const OpDev& op, bool trunc, const T* X, int64_t xms, int64_t xts, int ilo1,
                   int ihi1, int ilo2, int ihi2, int j0, int L, const T* base, ColMap bmap, T* out, ColMap omap,
                   double scale, int scale_off, double mean_c, int nvec, hipStream_t st);
// KKT apply with the general coupling; T1, T2: scratch of one field block per vector each.
template <typename T>
void launch_gen_kkt(const Shape& s, const OpDev& op, const T* x, T* y, T* T1, T* T2, int nvec, hipStream_t st);

// Chebyshev semi-iteration for the mass blocks (state + control) of nvec KKT vectors.
template <typename T>
void launch_mass_cheb(const Shape& s, const OpDev& op, const T* r, T* z, T* bufA, T* bufB,
                      int nvec, int steps, hipStream_t st);

// W = scale_col * M V  (column scale = tau * D_t * (1+gamma if j>0 else 1) * extra)
template <typename T>
void launch_mass_scaled(const Shape& s, const OpDev& op, const T* V, ColMap vmap, T* W, ColMap wmap,
                        int ncols, int nvec_members, hipStream_t st);

// Fused multigrid levels (mg.hip): down = npre pre-smoothing steps from zero +
// residual + restriction, the pre-smoothed iterate stored to xp; up = xp +
// prolongation of the coarse correction + npost post-smoothing steps.  Coarse
// arrays and xp are contiguous [column][(m/2+1)^2] and [column][(m+1)^2].
// Columns c with act != null and act[c / cpv] == 0 are skipped (cpv: columns
// per vector).
template <typename T>
void launch_mg_down(int m, const LevelDev* lev, int lvl, int npre, const T* b, ColMap bmap, T* bc, T* xp, int ncols,
                    int cpm, const int* act, int cpv, hipStream_t st);
template <typename T>
void launch_mg_up(int m, const LevelDev* lev, int lvl, int npost, const T* ec, const T* b, ColMap bmap, const T* xp,
                  T* xo, ColMap xomap, int ncols, int cpm, const int* act, int cpv, hipStream_t st);
template <typename T>
void launch_mg_tail(int m0, const LevelDev* lev, int lvl0, int npre, int npost, const T* b, ColMap bmap, T* x,
                    ColMap xmap, const T* ainv, int ncols, int cpm, const int* act, int cpv, hipStream_t st);

// All Chebyshev mass steps in one LDS-tiled kernel; false when steps > 9.
template <typename T>
bool launch_mass_cheb_fused(const Shape& s, const OpDev& op, const T* r, T* z, int nvec, int steps, hipStream_t st);
// The same on ngrp groups of ncols consecutive columns of [y | u] (n_t n_xi
// state columns, then the control columns; the block scalings of those
// columns), group g starting at column l0 + g * gstride, input and output
// with their own vector strides.
template <typename T>
bool launch_mass_cheb_cols(const Shape& s, const OpDev& op, const T* r, int64_t rstride, T* z, int64_t zstride, int l0,
                           int ncols, int ngrp, int gstride, int nvec, int steps, hipStream_t st);

// Exact solve by the 2D sine transform (dst.hip) on ncols columns:
// mode 1: x = (a1 K + b1 M)^{-1} b with the scalars of member c / cpm;
// mode 2: the mass blocks, x = f M^{-1} b with the column scale f of the
// Chebyshev mass kernels (columns of [y | u] of nt * nxi each per vector).
// sintab: sin(pi m / n), m < 2n; eig: [2][n+1] 1D stiffness / mass
// eigenvalues; s1, s2: FP64 scratch of ncols * (n+1)^2 each.
template <typename T>
void launch_dst_solve(int n, int mode, const MemberDev* mem, int shared, const double* sintab, const double* eig,
                      const T* b, ColMap bmap, T* x, ColMap xmap, int ncols, int cpm, int nt, int nxi, int time, double* s1,
                      double* s2, const int* act, int cpv, hipStream_t st);
// Richardson residual out = R - off_scale Y - b1 M V per column (member c / cpv).
template <typename T>
void launch_z_residual(int n, const T* R, ColMap rmap, const T* Y, const T* V, ColMap vmap, T* out, ColMap omap,
                       const MemberDev* mem, int ncols, int cpv, int shared, const int* act, hipStream_t st);
// out = A + B column by column.
template <typename T>
void launch_cols_add(int64_t nodes, const T* A, ColMap amap, const T* Bv, ColMap bmap, T* out, ColMap omap, int ncols,
                     int cpv, const int* act, hipStream_t st);

// Multigrid coarsest level: x = A_c^{-1} b (FP64 MFMA, FP32 plain).
template <typename T>
void launch_mg_coarse(const T* ainv, const T* bc, ColMap bmap, T* xc, ColMap xmap, int ncols,
                      int cols_per_member, hipStream_t st);

// BLAS-like kernels on flat vectors (FP64 Krylov arithmetic).
void launch_multidot(const double* V, int64_t vstride, int nv, const double* w, int64_t n,
                     int nmem, int64_t mstride, double* partial, int nblk, hipStream_t st);
void launch_cgs_update_dot(const double* V, int64_t vstride, int nv, const double* h, int hstride,
                           double* w, int64_t n, int nmem, int64_t mstride, double* partial,
                           int nblk, hipStream_t st);
void launch_cgs_update_norm(const double* V, int64_t vstride, int nv, const double* h, int hstride,
                            const double* w, double* out, int64_t n, int nmem, int64_t mstride,
                            double* partial, int nblk, hipStream_t st);
void launch_reduce_partials(const double* partial, int nblk, int nv, int nmem, double* out,
                            int out_stride, int out_offset, hipStream_t st);
void launch_scale_vec(double* v, const double* sdev, int sstride, int64_t n, int nmem,
                      int64_t mstride, hipStream_t st);
void launch_multi_axpy(const void* Z, int zfp32, int64_t zstride, int nv_max, const int* nv_mem,
                       const double* y, int ystride, double* x, int64_t n, int nmem,
                       int64_t mstride, hipStream_t st);
void launch_sub_norm(const double* b, double* r, int64_t n, int nmem, int64_t mstride,
                     double* partial, int nblk, hipStream_t st);   // r = b - r, partial ||r||^2
void launch_norm(const double* x, int64_t n, int nmem, int64_t mstride, double* partial, int nblk,
                 hipStream_t st);
void launch_axpby(double a, const double* x, double b, double* y, int64_t n, hipStream_t st);
void launch_cast_d2f(const double* x, float* y, int64_t n, hipStream_t st);
void launch_cast_f2d(const float* x, double* y, int64_t n, hipStream_t st);
template <typename TD>
void launch_copy_scale_rows(const double* src, TD* dst, const double* inv_norm, int64_t n,
                            int nmem, int64_t mstride, hipStream_t st);
template <typename T>
void launch_zero_ring(T* x, int n, int64_t ncols, hipStream_t st);
template <typename T>
void launch_fill_zero(T* x, int64_t count, hipStream_t st);   // x[0..count) = 0 (a kernel, capturable)

// Arnoldi bookkeeping on the device (one thread per member).
constexpr int kSlots = 64;   // partial-sum slots per member in Krylov reductions

struct KrylovDev {
    double* H;        // [member][(restart+1)][restart] column-major per member: H[i + j*(restart+1)]
    double* cs;       // [member][restart]
    double* sn;       // [member][restart]
    double* g;        // [member][restart+1]
    double* h1;       // [member][restart+1] first CGS pass coefficients
    double* h2;       // [member][restart+1] second pass coefficients
    double* nrm;      // [member] ||w2||^2 then 1/||w2||
    double* y;        // [member][restart]
    double* resid;    // [member] |g_{j+1}| (estimate)
    int* active;      // [member] 1 while iterating in the current cycle (cleared by k_conv_check)
    int* iters;       // [member] iterations so far (all cycles of the solve)
    const int* itmax; // [member] iteration limit
    int* jend;        // [member] iterations of the current cycle
    const double* tol;   // [member] stop when the estimate reaches this
    double* dots;     // [member][kSlots] reduced dot products of the current pass (DCGS2)
    double* scal;     // [member][4] -, -, 1/nu, nu of the current candidate (DCGS2)
    double* R;        // [member][(restart+1)^2] U = V R, upper triangular, column-major (DCGS2)
    double* coef;     // [member][kSlots] update-pass coefficients s = R^{-1} [t; c] (DCGS2)
    int* pending;     // [member] 1 while the last Hessenberg column awaits its reorthogonalisation
};
void launch_arnoldi_finish(KrylovDev k, int restart, int j, int nmem, hipStream_t st);
// DCGS2 passes over a basis stored in TV (double, or float in the FP32
// inner cycles of iterative refinement); sums are formed in double.
template <typename TV>
void launch_dcgs_dots(const TV* V, int64_t vstride, int nv, const TV* w, int64_t n, int nmem,
                      int64_t mstride, const int* active, const int* pending, double* partial, int nblk,
                      hipStream_t st);
template <typename TV>
void launch_dcgs_update(TV* V, int64_t vstride, int nv, const TV* w, int64_t n, int nmem, int64_t mstride,
                        const double* coef, const double* scal, const int* active, int nblk, hipStream_t st);
void launch_dcgs_finish(KrylovDev k, int restart, int j, int mode, int nmem, hipStream_t st);
void launch_cycle_start(KrylovDev k, int restart, const double* beta0, int nmem, hipStream_t st);
void launch_back_solve(KrylovDev k, int restart, const int* jend, int nmem, hipStream_t st);
// End of iteration j: every active member counts the iteration (jend = j + 1,
// iters + 1) and stops once its estimate reaches tol or iters reaches itmax.
// Launched after the iteration's last pass, so every pass of iteration j saw
// the flags of its start.
void launch_conv_check(KrylovDev k, int j, int nmem, hipStream_t st);

}  // namespace sg
