// HIP kernels for gfx950 (MI355X): the stochastic-Galerkin operator and KKT
// applies, the hierarchical Gauss-Seidel right-hand sides, Chebyshev mass
// solves, geometric multigrid and the FP64 Krylov vector arithmetic.
//
// All stencils are Q1 on the uniform n x n grid of [0,1]^2 (h = 1/n), node
// (ix, iy) at flat index iy*(n+1)+ix, element (ex, ey) at ey*n+ex.
//   unit stiffness K (constant coefficient): centre 8/3, eight neighbours -1/3
//   mass M_h: (h^2/36) [16 centre, 4 edge, 1 corner]
//   stiffness of a per-element coefficient c_e at node p:
//     (1/6) sum_{e contains p} c_e (4 x_p - x_h(e) - x_v(e) - 2 x_d(e))
//   with h, v, d the horizontal, vertical and diagonal partners of p in e.
// Boundary nodes are Dirichlet (eliminated): outputs write 0 there and inputs
// read there are treated as 0.
#include "common.hpp"

namespace sg {

namespace {

constexpr int TX = 64;   // nodes per block row (one wavefront)
constexpr int TY = 4;    // block rows

template <typename T>
struct Nine {
    T c, w, e, s, n, sw, se, nw, ne;
};

// Load the 3x3 neighbourhood of interior node (ix, iy); neighbours on the
// boundary ring read as zero.
// Values are widened to FP64 (the SG stencils compute in FP64 whatever the
// storage type).
template <typename T>
__device__ __forceinline__ Nine<double> load9(const T* __restrict__ x, int n, int ix, int iy) {
    const int N1 = n + 1;
    const int64_t p = (int64_t)iy * N1 + ix;
    const bool w = ix > 1, e = ix < n - 1, s = iy > 1, nn = iy < n - 1;
    Nine<double> v;
    v.c = (double)x[p];
    v.w = w ? (double)x[p - 1] : 0.0;
    v.e = e ? (double)x[p + 1] : 0.0;
    v.s = s ? (double)x[p - N1] : 0.0;
    v.n = nn ? (double)x[p + N1] : 0.0;
    v.sw = (s && w) ? (double)x[p - N1 - 1] : 0.0;
    v.se = (s && e) ? (double)x[p - N1 + 1] : 0.0;
    v.nw = (nn && w) ? (double)x[p + N1 - 1] : 0.0;
    v.ne = (nn && e) ? (double)x[p + N1 + 1] : 0.0;
    return v;
}

template <typename T>
__device__ __forceinline__ void axpy9(Nine<T>& a, T g, const Nine<T>& b) {
    a.c += g * b.c; a.w += g * b.w; a.e += g * b.e; a.s += g * b.s; a.n += g * b.n;
    a.sw += g * b.sw; a.se += g * b.se; a.nw += g * b.nw; a.ne += g * b.ne;
}

template <typename T>
__device__ __forceinline__ Nine<T> scale9(T g, const Nine<T>& b) {
    Nine<T> a;
    a.c = g * b.c; a.w = g * b.w; a.e = g * b.e; a.s = g * b.s; a.n = g * b.n;
    a.sw = g * b.sw; a.se = g * b.se; a.nw = g * b.nw; a.ne = g * b.ne;
    return a;
}

template <typename T>
__device__ __forceinline__ T unit_stiff(const Nine<T>& v) {
    return T(8.0 / 3.0) * v.c - T(1.0 / 3.0) * (v.w + v.e + v.s + v.n + v.sw + v.se + v.nw + v.ne);
}

template <typename T>
__device__ __forceinline__ T mass9(const Nine<T>& v, T h2_36) {
    return h2_36 * (T(16) * v.c + T(4) * (v.w + v.e + v.s + v.n) + (v.sw + v.se + v.nw + v.ne));
}

// Stiffness with per-element coefficients c (plane [ey][ex] of one mode).
template <typename T>
__device__ __forceinline__ T var_stiff(const T* __restrict__ c, int n, int ix, int iy, const Nine<T>& v) {
    const T cSW = c[(iy - 1) * n + ix - 1], cSE = c[(iy - 1) * n + ix];
    const T cNW = c[iy * n + ix - 1], cNE = c[iy * n + ix];
    T s = T(4) * v.c * ((cSW + cSE) + (cNW + cNE));
    s -= v.w * (cSW + cNW) + v.e * (cSE + cNE) + v.s * (cSW + cSE) + v.n * (cNW + cNE);
    s -= T(2) * (cSW * v.sw + cSE * v.se + cNW * v.nw + cNE * v.ne);
    return s * T(1.0 / 6.0);
}

// (A X)_j at interior node (ix, iy) for one (member, t) block X [j][node]:
//   c0 K_unit X_j + sum_{k in mask} K_k (g- X_{j-e_k} + g+ X_{j+e_k})
template <typename T>
__device__ __forceinline__ double sg_node(const T* __restrict__ X, int64_t nodes, int j, int n, int ix, int iy,
                                          int M, const int32_t* __restrict__ nidx,
                                          const double* __restrict__ nval, const double* __restrict__ coef,
                                          int64_t cplane, double c0, bool with_mean, uint32_t mask,
                                          bool lower, bool upper) {
    double acc = 0.0;
    if (with_mean) acc = c0 * unit_stiff(load9(X + (int64_t)j * nodes, n, ix, iy));
    for (int k = 1; k <= M; ++k) {
        if (!((mask >> (k - 1)) & 1u)) continue;
        const int base = (j * M + (k - 1)) * 2;
        const int im = lower ? nidx[base] : -1;
        const int ip = upper ? nidx[base + 1] : -1;
        if (im < 0 && ip < 0) continue;
        Nine<double> w;
        if (im >= 0) {
            w = scale9(nval[base], load9(X + (int64_t)im * nodes, n, ix, iy));
            if (ip >= 0) axpy9(w, nval[base + 1], load9(X + (int64_t)ip * nodes, n, ix, iy));
        } else {
            w = scale9(nval[base + 1], load9(X + (int64_t)ip * nodes, n, ix, iy));
        }
        acc += var_stiff(coef + (int64_t)k * cplane, n, ix, iy, w);
    }
    return acc;
}

__device__ __forceinline__ int node_x() { return blockIdx.x % 0x7fffffff; }

// Map a flat tile index to (ix0, iy0) tiles of TX x TY nodes.
__device__ __forceinline__ void tile_coords(int n, int tile, int& ix, int& iy) {
    const int tiles_x = (n + 1 + TX - 1) / TX;
    ix = (tile % tiles_x) * TX + threadIdx.x % TX;
    iy = (tile / tiles_x) * TY + threadIdx.x / TX;
}

constexpr int kJChunk = 8;

// --------------------------------------------------------------------------
// SG operator apply: y = A x for each (vector, t) block.
// grid: x = node tiles, y = chaos chunks, z = nvec*nt slices.
// --------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_sg_apply(int n, int M, int nxi, int nt, int64_t nodes,
                                                  OpDev op, const T* __restrict__ x, T* __restrict__ y, uint32_t mask) {
    int ix, iy;
    tile_coords(n, blockIdx.x, ix, iy);
    if (ix > n || iy > n) return;
    const int slice = blockIdx.z;
    const int vec = slice / nt;
    const int mem = op.mem_shared ? 0 : vec;
    const int64_t off = (int64_t)slice * nxi * nodes;
    const T* X = x + off;
    T* Y = y + off;
    const double* coef = op.coef64 + (int64_t)mem * op.coef_mstride;
    const int64_t cplane = (int64_t)n * n;
    const double c0 = op.mem[mem].c0;
    const bool interior = ix > 0 && ix < n && iy > 0 && iy < n;
    const int64_t p = (int64_t)iy * (n + 1) + ix;
    const int j0 = blockIdx.y * kJChunk;
    const int j1 = min(nxi, j0 + kJChunk);
    for (int j = j0; j < j1; ++j) {
        double v = 0.0;
        if (interior)
            v = sg_node<T>(X, nodes, j, n, ix, iy, M, op.nbr_idx, op.nbr_val, coef, cplane, c0, true,
                           mask, true, true);
        Y[(int64_t)j * nodes + p] = (T)v;
    }
}

// --------------------------------------------------------------------------
// Fused KKT apply.  Steady (eq. stoch-system, matricized eq. stoch-system-m with A_l):
//   R^Y = M Y H^gamma - A Lambda;  R^U = beta M U + M Lambda;  R^L = -A Y + M U.
// Time (eq. KKT:stoch-time-dependent), L = M-cal + tau A, D = diag(1/2,1..1,1/2):
//   R^Y_t = tau D_t M_gamma Y_t - (M L_t + tau A L_t) + M L_{t+1}
//   R^U_t = beta tau D_t M U_t + tau M L_t
//   R^L_t = -(M Y_t + tau A Y_t) + M Y_{t-1} + tau M U_t
// grid: x = node tiles, y = chaos chunks, z = nvec*nt.
// --------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_kkt_apply(int n, int M, int nxi, int nt, int time, int64_t nodes,
                                                   OpDev op, const T* __restrict__ x, T* __restrict__ y) {
    int ix, iy;
    tile_coords(n, blockIdx.x, ix, iy);
    if (ix > n || iy > n) return;
    const int slice = blockIdx.z;
    const int vec = slice / nt;
    if (op.active && !op.active[vec]) return;
    const int t = slice % nt;
    const int mem = op.mem_shared ? 0 : vec;
    const int64_t blk = (int64_t)nt * nxi * nodes;
    const int64_t tst = (int64_t)nxi * nodes;
    const T* Yv = x + (int64_t)vec * 3 * blk;
    const T* Uv = Yv + blk;
    const T* Lv = Uv + blk;
    T* RY = y + (int64_t)vec * 3 * blk;
    T* RU = RY + blk;
    T* RL = RU + blk;
    const MemberDev md = op.mem[mem];
    const double* coef = op.coef64 + (int64_t)mem * op.coef_mstride;
    const int64_t cplane = (int64_t)n * n;
    const double c0 = md.c0;
    const double h = 1.0 / (double)n;
    const double h2_36 = h * h / 36.0;
    const bool interior = ix > 0 && ix < n && iy > 0 && iy < n;
    const int64_t p = (int64_t)iy * (n + 1) + ix;
    const double tau = md.tau;
    const double Dt = (time && (t == 0 || t == nt - 1)) ? 0.5 : 1.0;
    const double beta = md.beta;
    const double hg = md.hg;
    const int j0 = blockIdx.y * kJChunk;
    const int j1 = min(nxi, j0 + kJChunk);
    const T* Yt = Yv + t * tst;
    const T* Ut = Uv + t * tst;
    const T* Lt = Lv + t * tst;
    for (int j = j0; j < j1; ++j) {
        const int64_t q = (int64_t)j * nodes + p;
        double ry = 0.0, ru = 0.0, rl = 0.0;
        if (interior) {
            const double AY = sg_node<T>(Yt, nodes, j, n, ix, iy, M, op.nbr_idx, op.nbr_val, coef, cplane, c0,
                                         true, 0xffffffffu, true, true);
            const double AL = sg_node<T>(Lt, nodes, j, n, ix, iy, M, op.nbr_idx, op.nbr_val, coef, cplane, c0,
                                         true, 0xffffffffu, true, true);
            const double MY = mass9(load9(Yt + (int64_t)j * nodes, n, ix, iy), h2_36);
            const double MU = mass9(load9(Ut + (int64_t)j * nodes, n, ix, iy), h2_36);
            const double ML = mass9(load9(Lt + (int64_t)j * nodes, n, ix, iy), h2_36);
            const double hgj = j == 0 ? 1.0 : hg;
            if (!time) {
                ry = hgj * MY - AL;
                ru = beta * MU + ML;
                rl = MU - AY;
            } else {
                double MLn = 0.0, MYp = 0.0;
                if (t + 1 < nt) MLn = mass9(load9(Lt + tst + (int64_t)j * nodes, n, ix, iy), h2_36);
                if (t > 0) MYp = mass9(load9(Yt - tst + (int64_t)j * nodes, n, ix, iy), h2_36);
                ry = tau * Dt * hgj * MY - (ML + tau * AL) + MLn;
                ru = beta * tau * Dt * MU + tau * ML;
                rl = -(MY + tau * AY) + MYp + tau * MU;
            }
        }
        RY[t * tst + q] = (T)ry;
        RU[t * tst + q] = (T)ru;
        RL[t * tst + q] = (T)rl;
    }
}

// --------------------------------------------------------------------------
// hGS off-level right-hand side for degree level d (Algorithm 1, eq. alg-hGS2
// with the affine coupling: the lower level contributes E, the upper F).
// grid: x = node tiles, y = level-column chunks, z = nmembers*nt.
// --------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_hgs_rhs(int n, int M, int nxi, int nt, int64_t nodes, OpDev op,
                                                 int j0lvl, int L, uint32_t mask, int lower, int upper,
                                                 const T* __restrict__ base, ColMap bmap,
                                                 const T* __restrict__ V, ColMap vmap,
                                                 T* __restrict__ out, ColMap omap) {
    int ix, iy;
    tile_coords(n, blockIdx.x, ix, iy);
    if (ix > n || iy > n) return;
    const int slice = blockIdx.z;           // member*nt + t
    const int mem_i = slice / nt;
    if (op.active && !op.active[mem_i]) return;
    const int t = slice % nt;
    const int mem = op.mem_shared ? 0 : mem_i;
    const double* coef = op.coef64 + (int64_t)mem * op.coef_mstride;
    const int64_t cplane = (int64_t)n * n;
    const double scale = op.off_sign * op.mem[mem].off_scale;
    const bool interior = ix > 0 && ix < n && iy > 0 && iy < n;
    const int64_t p = (int64_t)iy * (n + 1) + ix;
    const T* Vb = V + (int64_t)mem_i * vmap.mstride + (int64_t)t * vmap.tstride;
    const int l0 = blockIdx.y * kJChunk;
    const int l1 = min(L, l0 + kJChunk);
    for (int l = l0; l < l1; ++l) {
        const int c = slice * L + l;
        const int j = j0lvl + l;
        double v = 0.0;
        if (interior) {
            v = (double)base[bmap.off(c) + p];
            if (mask)
                v -= scale * sg_node<T>(Vb, vmap.nodes, j, n, ix, iy, M, op.nbr_idx, op.nbr_val, coef, cplane,
                                        0.0, false, mask, lower != 0, upper != 0);
        }
        out[omap.off(c) + p] = (T)v;
    }
}

// --------------------------------------------------------------------------
// Chebyshev semi-iteration on the mass matrix (Golub-Varga), state and
// control blocks.  D = 1.25 diag(M) = 1.25 * 4h^2/9, rho = 0.8.
// Column l of a vector's first 2*nt*nxi columns: var = l / (nt*nxi),
// t = (l / nxi) % nt, j = l % nxi; final scale 1/(hg_j tau D_t) for the
// state, 1/(beta tau D_t) for the control (tau = D_t = 1 when steady).
// --------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_mass_cheb_step(int n, int nxi, int nt, int time, int64_t nodes,
                                                        OpDev op, int64_t vstride, const T* __restrict__ r,
                                                        const T* __restrict__ xk, const T* __restrict__ xkm1,
                                                        T* __restrict__ xout, T omega, int first, int last) {
    int ix, iy;
    tile_coords(n, blockIdx.x, ix, iy);
    if (ix > n || iy > n) return;
    const int vec = blockIdx.z;
    if (op.active && !op.active[vec]) return;
    const int mem = op.mem_shared ? 0 : vec;
    const int64_t p = (int64_t)iy * (n + 1) + ix;
    const bool interior = ix > 0 && ix < n && iy > 0 && iy < n;
    const T h = T(1) / T(n);
    const T h2_36 = h * h / T(36);
    const T dinv = T(1) / (T(1.25) * T(4) * h * h / T(9));
    const int ncols = 2 * nt * nxi;
    const int l0 = blockIdx.y * kJChunk;
    const int l1 = min(ncols, l0 + kJChunk);
    const MemberDev md = op.mem[mem];
    for (int l = l0; l < l1; ++l) {
        const int64_t q = (int64_t)vec * vstride + (int64_t)l * nodes + p;       // r / out addressing (KKT vector)
        const int64_t qs = ((int64_t)vec * ncols + l) * nodes + p;                // scratch addressing
        T v = T(0);
        if (interior) {
            const T b = r[q];
            if (first) {
                v = dinv * b;
            } else {
                const T res = b - (T)mass9(load9(xk + ((int64_t)vec * ncols + l) * nodes, n, ix, iy), (double)h2_36);
                v = omega * (dinv * res + xk[qs] - xkm1[qs]) + xkm1[qs];
            }
            if (last) {
                const int var = l / (nt * nxi);
                const int t = (l / nxi) % nt;
                const int j = l % nxi;
                const T Dt = (time && (t == 0 || t == nt - 1)) ? T(0.5) : T(1);
                const T tau = T(md.tau);
                const T s = var == 0 ? (j == 0 ? T(1) : T(md.hg)) : T(md.beta);
                v = v / (s * tau * Dt);
            }
        }
        if (last)
            xout[q] = v;
        else
            xout[qs] = v;
    }
}

// W = tau D_t (1 or hg) M V on the columns of a field block (Schur block middle
// factor).  A wavefront owns one column; each of its 32-lane halves computes
// kMassRows node rows of a 30-node-wide tile (lanes 0 and 31 are halos): every
// node value is loaded once per strip (plus two halo rows) and its x
// neighbours come from one left and one right lane shuffle per row.  Values on
// the boundary ring read as zero.
constexpr int kMassRows = 8;
template <typename T>
__global__ __launch_bounds__(256) void k_mass_scaled(int n, int nt, int time, OpDev op, const T* __restrict__ V,
                                                     ColMap vmap, T* __restrict__ W, ColMap wmap, int ncols,
                                                     int tiles_x) {
    constexpr int R = kMassRows;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int c = blockIdx.y * 4 + wave;
    if (c >= ncols) return;                          // uniform per wavefront; no barriers below
    if (op.active && !op.active[vmap.member(c)]) return;
    const int tx = blockIdx.x % tiles_x, ty = blockIdx.x / tiles_x;
    const int lane = threadIdx.x & 63;
    const int gl = lane & 31, grp = lane >> 5;
    const int X = tx * 30 + gl - 1;
    const int y0 = (ty * 2 + grp) * R;               // output rows y0 .. y0+R-1
    const int N1 = n + 1;
    const int xc = min(max(X, 0), n);
    const bool xin = X >= 1 && X <= n - 1;
    const T* v = V + vmap.off(c);
    T rc[R + 2], rl[R + 2], rr[R + 2];
    // all row loads first, masked afterwards (a select next to each load lets
    // the compiler branch around it and wait for every load in turn)
#pragma unroll
    for (int k = 0; k < R + 2; ++k) rc[k] = v[(int64_t)min(max(y0 - 1 + k, 0), n) * N1 + xc];
#pragma unroll
    for (int k = 0; k < R + 2; ++k) {
        const int Y = y0 - 1 + k;
        rc[k] = (xin && Y >= 1 && Y <= n - 1) ? rc[k] : T(0);
    }
#pragma unroll
    for (int k = 0; k < R + 2; ++k) {
        rl[k] = __shfl_up(rc[k], 1, 32);
        rr[k] = __shfl_down(rc[k], 1, 32);
    }
    const int mem_i = vmap.member(c);
    const int mem = op.mem_shared ? 0 : mem_i;
    const MemberDev md = op.mem[mem];
    const int t = vmap.tstep(c);
    const int j = vmap.chaos(c);
    const T Dt = (time && (t == 0 || t == nt - 1)) ? T(0.5) : T(1);
    const T sc = T(md.tau) * Dt * (j == 0 ? T(1) : T(md.hg));
    const T h = T(1) / T(n);
    const T h2_36 = h * h / T(36);
    T* w = W + wmap.off(c);
    const bool xout = gl >= 1 && gl <= 30 && X <= n;
#pragma unroll
    for (int k = 1; k <= R; ++k) {
        const int Y = y0 - 1 + k;
        if (xout && Y <= n) {
            const bool inter = xin && Y >= 1 && Y <= n - 1;
            const T m9 = h2_36 * (T(16) * rc[k] + T(4) * (rl[k] + rr[k] + rc[k - 1] + rc[k + 1]) +
                                  (rl[k - 1] + rr[k - 1] + rl[k + 1] + rr[k + 1]));
            w[(int64_t)Y * N1 + X] = inter ? sc * m9 : T(0);
        }
    }
}

// --------------------------------------------------------------------------
// Multigrid coarsest level (the smoothing levels are in mg.hip).
// --------------------------------------------------------------------------
// Coarse solve x = A_c^{-1} b on the 8x8 grid (49 unknowns padded to 64) with
// FP64 MFMA 16x16x4 tiles: one wavefront computes a 64 x 16 block of
// x = Ainv (64 x 64) * B (64 x 16 columns of one member).
__global__ __launch_bounds__(64) void k_mg_coarse_f64(const double* __restrict__ ainv, const double* __restrict__ b,
                                                      ColMap bmap, double* __restrict__ x, ColMap xmap, int ncols,
                                                      int cpm) {
    typedef double v4d __attribute__((ext_vector_type(4)));
    const int lane = threadIdx.x;
    const int mem = blockIdx.y;
    const int c_begin = mem * cpm + blockIdx.x * 16;
    const int c_end = min((mem + 1) * cpm, ncols);
    if (c_begin >= c_end) return;
    const double* A = ainv + (int64_t)mem * kCoarsePad * kCoarsePad;
    const int col = lane % 16;
    const int kq = lane / 16;
    const int c = c_begin + col;
    const bool cvalid = c < c_end;
    const int N1 = kCoarseN + 1;
    v4d acc[4];
    for (int rt = 0; rt < 4; ++rt) acc[rt] = v4d{0.0, 0.0, 0.0, 0.0};
    for (int kb = 0; kb < kCoarsePad; kb += 4) {
        const int k = kb + kq;                                   // unknown index 0..63
        double bv = 0.0;
        if (cvalid && k < (kCoarseN - 1) * (kCoarseN - 1)) {
            const int ix = k % (kCoarseN - 1) + 1, iy = k / (kCoarseN - 1) + 1;
            bv = b[bmap.off(c) + iy * N1 + ix];
        }
        for (int rt = 0; rt < 4; ++rt) {
            const double av = A[(rt * 16 + col) * kCoarsePad + k];   // A[row = rt*16 + lane%16][k]
            acc[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[rt], 0, 0, 0);
        }
    }
    // acc[rt][i] holds row rt*16 + lane/16 + 4*i, column lane%16 (FP64 16x16x4 output layout)
    if (cvalid) {
        double* xo = x + xmap.off(c);
        for (int rt = 0; rt < 4; ++rt) {
            for (int i = 0; i < 4; ++i) {
                const int row = rt * 16 + kq + 4 * i;
                if (row < (kCoarseN - 1) * (kCoarseN - 1)) {
                    const int ix = row % (kCoarseN - 1) + 1, iy = row / (kCoarseN - 1) + 1;
                    xo[iy * N1 + ix] = acc[rt][i];
                }
            }
        }
        // boundary ring of the coarse column
        for (int q = kq; q < N1 * N1; q += 4) {
            const int ix = q % N1, iy = q / N1;
            if (ix == 0 || iy == 0 || ix == kCoarseN || iy == kCoarseN) xo[q] = 0.0;
        }
    }
}

// FP32 coarse solve (plain FMA; the FP32 path has no FP64 MFMA operand type).
__global__ __launch_bounds__(64) void k_mg_coarse_f32(const float* __restrict__ ainv, const float* __restrict__ b,
                                                      ColMap bmap, float* __restrict__ x, ColMap xmap, int ncols,
                                                      int cpm) {
    const int mem = blockIdx.y;
    const int c = mem * cpm + blockIdx.x;
    if (blockIdx.x >= cpm || c >= ncols) return;
    const float* A = ainv + (int64_t)mem * kCoarsePad * kCoarsePad;
    const int N1 = kCoarseN + 1;
    const int nu = (kCoarseN - 1) * (kCoarseN - 1);
    __shared__ float bs[kCoarsePad];
    const int lane = threadIdx.x;
    const float* bc = b + bmap.off(c);
    if (lane < nu) {
        const int ix = lane % (kCoarseN - 1) + 1, iy = lane / (kCoarseN - 1) + 1;
        bs[lane] = bc[iy * N1 + ix];
    }
    __syncthreads();
    float* xo = x + xmap.off(c);
    if (lane < nu) {
        float s = 0.f;
        for (int k = 0; k < nu; ++k) s += A[lane * kCoarsePad + k] * bs[k];
        const int ix = lane % (kCoarseN - 1) + 1, iy = lane / (kCoarseN - 1) + 1;
        xo[iy * N1 + ix] = s;
    }
    for (int q = lane; q < N1 * N1; q += 64) {
        const int ix = q % N1, iy = q / N1;
        if (ix == 0 || iy == 0 || ix == kCoarseN || iy == kCoarseN) xo[q] = 0.f;
    }
}

template <typename T>
__global__ void k_fill_zero(T* x, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        x[i] = T(0);
}

template <typename T>
__global__ void k_zero_ring(T* x, int n, int64_t ncols) {
    const int64_t nodes = (int64_t)(n + 1) * (n + 1);
    const int64_t per = 4 * (int64_t)n;
    const int64_t total = per * ncols;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = i / per;
        const int q = (int)(i % per);
        int ix, iy;
        if (q < n) { ix = q; iy = 0; }
        else if (q < 2 * n) { ix = n; iy = q - n; }
        else if (q < 3 * n) { ix = n - (q - 2 * n); iy = n; }
        else { ix = 0; iy = n - (q - 3 * n); }
        x[c * nodes + (int64_t)iy * (n + 1) + ix] = T(0);
    }
}

// --------------------------------------------------------------------------
// FP64 Krylov vector arithmetic.  Reductions are deterministic: each member's
// vector is split into `nblk` fixed chunks, block partials are written to
// memory and summed in a fixed order by k_reduce_partials.
// --------------------------------------------------------------------------
constexpr int RB = 256;      // threads per reduction block
constexpr int MAXV = 32;     // basis vectors per multi-vector launch
// partial sums: partial[(mem*kSlots + slot)*nblk + blk] (kSlots per member)

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block-reduce the first `nv` of NA per-thread accumulators into
// partial[(mem*nvmax + i)*nblk + blk].
template <int NA>
__device__ __forceinline__ void block_reduce_store(const double* acc, int nv, double* partial, int mem, int nvmax,
                                                   int nblk) {
    __shared__ double red[RB / 64][kSlots + 1];
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
#pragma unroll
    for (int i = 0; i < NA; ++i) {
        if (i < nv) {
            const double s = wave_sum(acc[i]);
            if (lane == 0) red[wave][i] = s;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < nv) {
        double s = 0.0;
        for (int w = 0; w < RB / 64; ++w) s += red[w][threadIdx.x];
        partial[((int64_t)mem * nvmax + threadIdx.x) * nblk + blockIdx.x] = s;
    }
}

__device__ __forceinline__ void chunk_range(int64_t n, int nblk, int blk, int64_t& lo, int64_t& hi) {
    const int64_t per = (n + nblk - 1) / nblk;
    lo = (int64_t)blk * per;
    hi = lo + per < n ? lo + per : n;
}

// Basis vectors are streamed once per pass and are far larger than the
// caches, so their loads bypass them.
__device__ __forceinline__ double ld_stream(const double* p) { return __builtin_nontemporal_load(p); }

// partial[i] = V_i . w  (i < nv <= NV).  Two elements per thread per trip keep
// 2*nv loads in flight per lane.
template <int NV>
__global__ __launch_bounds__(RB) void k_multidot(const double* __restrict__ V, int64_t vstride, int nv,
                                                 const double* __restrict__ w, int64_t n, int64_t mstride,
                                                 double* __restrict__ partial, int nblk) {
    const int mem = blockIdx.y;
    int64_t lo, hi;
    chunk_range(n, nblk, blockIdx.x, lo, hi);
    double acc[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = 0.0;
    const double* wm = w + mem * mstride;
    const double* Vm = V + mem * mstride;
    int64_t e = lo + threadIdx.x;
    for (; e + RB < hi; e += 2 * RB) {
        const double w0 = ld_stream(wm + e), w1 = ld_stream(wm + e + RB);
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            if (i < nv) {
                const double* p = Vm + i * vstride + e;
                acc[i] += ld_stream(p) * w0;
                acc[i] += ld_stream(p + RB) * w1;
            }
        }
    }
    if (e < hi) {
        const double we = wm[e];
#pragma unroll
        for (int i = 0; i < NV; ++i)
            if (i < nv) acc[i] += Vm[i * vstride + e] * we;
    }
    block_reduce_store<NV>(acc, nv, partial, mem, kSlots, nblk);
}

// w1 = w - sum_i h_i V_i (written to w), partial[i] = V_i . w1
template <int NV>
__global__ __launch_bounds__(RB) void k_cgs_update_dot(const double* __restrict__ V, int64_t vstride, int nv,
                                                       const double* __restrict__ h, int hstride,
                                                       double* __restrict__ w, int64_t n, int64_t mstride,
                                                       double* __restrict__ partial, int nblk) {
    const int mem = blockIdx.y;
    int64_t lo, hi;
    chunk_range(n, nblk, blockIdx.x, lo, hi);
    double hc[NV], acc[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        hc[i] = i < nv ? h[mem * hstride + i] : 0.0;
        acc[i] = 0.0;
    }
    double* wm = w + mem * mstride;
    const double* Vm = V + mem * mstride;
    for (int64_t e = lo + threadIdx.x; e < hi; e += RB) {
        double v[NV];
        double we = wm[e];
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            v[i] = i < nv ? ld_stream(Vm + i * vstride + e) : 0.0;
            we -= hc[i] * v[i];
        }
        wm[e] = we;
#pragma unroll
        for (int i = 0; i < NV; ++i) acc[i] += v[i] * we;
    }
    block_reduce_store<NV>(acc, nv, partial, mem, kSlots, nblk);
}

// out = w - sum_i h_i V_i, partial[0] = ||out||^2
template <int NV>
__global__ __launch_bounds__(RB) void k_cgs_update_norm(const double* __restrict__ V, int64_t vstride, int nv,
                                                        const double* __restrict__ h, int hstride,
                                                        const double* __restrict__ w, double* __restrict__ out,
                                                        int64_t n, int64_t mstride, double* __restrict__ partial,
                                                        int nblk) {
    const int mem = blockIdx.y;
    int64_t lo, hi;
    chunk_range(n, nblk, blockIdx.x, lo, hi);
    double hc[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) hc[i] = i < nv ? h[mem * hstride + i] : 0.0;
    double acc[1] = {0.0};
    const double* wm = w + mem * mstride;
    double* om = out + mem * mstride;
    const double* Vm = V + mem * mstride;
    for (int64_t e = lo + threadIdx.x; e < hi; e += RB) {
        double we = wm[e];
#pragma unroll
        for (int i = 0; i < NV; ++i)
            if (i < nv) we -= hc[i] * ld_stream(Vm + i * vstride + e);
        om[e] = we;
        acc[0] += we * we;
    }
    block_reduce_store<1>(acc, 1, partial, mem, kSlots, nblk);
}

// ---- Arnoldi with delayed reorthogonalization (DCGS2) ----
// Slot j of the basis holds the candidate u_j (one Gram-Schmidt pass, scaled
// by an estimate of its norm) and is never rewritten: the orthonormal basis is
// V = U R^{-1}, applied through R by the bookkeeping kernel (k_dcgs_finish).
//
constexpr int kDotsU = 4;   // 16-byte groups per lane per trip, dots pass
constexpr int kUpdU = 8;    // 16-byte groups per lane per trip, update pass

// The basis (and w) are stored in TV = double or float; every product and
// sum is formed in double.  A member's vector is read in 16-byte groups of
// GW = 16 / sizeof(TV) consecutive elements, counted from the member's first
// element: with AL the group is 16-byte aligned and read by one load, else
// element by element (same arithmetic either way, so a member's sums do not
// depend on where the batch places it).  A group is held as GW doubles.
template <typename TV>
struct Grp {
    static constexpr int GW = 16 / (int)sizeof(TV);
    double v[GW];
};
typedef double dbl2 __attribute__((ext_vector_type(2)));
typedef float flt4 __attribute__((ext_vector_type(4)));

template <bool AL, bool NT, typename TV>
__device__ __forceinline__ Grp<TV> ld_grp(const TV* base, int64_t p) {
    Grp<TV> g;
    constexpr int GW = Grp<TV>::GW;
    if (AL) {
        if constexpr (sizeof(TV) == 8) {
            const dbl2* q = reinterpret_cast<const dbl2*>(base) + p;
            const dbl2 x = NT ? __builtin_nontemporal_load(q) : *q;
            g.v[0] = x.x;
            g.v[1] = x.y;
        } else {
            const flt4* q = reinterpret_cast<const flt4*>(base) + p;
            const flt4 x = NT ? __builtin_nontemporal_load(q) : *q;
            g.v[0] = x.x;
            g.v[1] = x.y;
            g.v[2] = x.z;
            g.v[3] = x.w;
        }
    } else {
        const TV* q = base + GW * p;
#pragma unroll
        for (int u = 0; u < GW; ++u) g.v[u] = (double)(NT ? __builtin_nontemporal_load(q + u) : q[u]);
    }
    return g;
}
template <bool AL, typename TV>
__device__ __forceinline__ void st_grp(TV* base, int64_t p, const Grp<TV>& g) {
    constexpr int GW = Grp<TV>::GW;
    if (AL) {
        if constexpr (sizeof(TV) == 8)
            reinterpret_cast<dbl2*>(base)[p] = dbl2{g.v[0], g.v[1]};
        else
            reinterpret_cast<flt4*>(base)[p] = flt4{(float)g.v[0], (float)g.v[1], (float)g.v[2], (float)g.v[3]};
    } else {
#pragma unroll
        for (int u = 0; u < GW; ++u) base[GW * p + u] = (TV)g.v[u];
    }
}
template <typename TV>
__device__ __forceinline__ double grp_dot(const Grp<TV>& a, const Grp<TV>& b) {
    double s = a.v[0] * b.v[0];
#pragma unroll
    for (int u = 1; u < Grp<TV>::GW; ++u) s += a.v[u] * b.v[u];
    return s;
}

// Dots pass, with w: slots [0, nv) a_i = V_i.u, [nv, 2nv) t_i = V_i.w,
// 2nv: u.u, 2nv+1: u.w, 2nv+2: w.w; without w: [0, nv) a_i, nv: u.u.
// u is basis slot nv.  The block's four wavefronts split the basis vectors
// (vector i goes to wavefront i mod 4, at most NPW each) and each walks the
// block's whole chunk of element groups, so a lane carries at most 2 NPW + 1
// sums and keeps many loads in flight; u and w are re-read by the four
// wavefronts from cache.  Members with neither flag set are skipped.
template <int NPW, bool WITH_W, bool AL, typename TV>
__device__ __forceinline__ void dcgs_dots_body(const TV* __restrict__ V, int64_t vstride, int nv,
                                               const TV* __restrict__ w, int64_t n, int64_t mstride,
                                               double* __restrict__ partial, int nblk) {
    constexpr int GW = Grp<TV>::GW;
    const int mem = blockIdx.y;
    int64_t lo, hi;
    chunk_range(n / GW, nblk, blockIdx.x, lo, hi);      // group range
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    // the wavefront's scalar product: wave 1 u.u (also without w), wave 2 u.w, wave 3 w.w
    const int sdot = WITH_W ? wave : (wave == 1 ? 1 : 0);
    constexpr int NA = WITH_W ? 2 * NPW + 1 : NPW + 1;
    double acc[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) acc[i] = 0.0;
    const TV* Vm = V + mem * mstride;
    const TV* um = Vm + nv * vstride;
    const TV* wm = WITH_W ? w + mem * mstride : um;
    auto add = [&](const Grp<TV>* ue, const Grp<TV>* we, int cnt) {
        for (int u = 0; u < cnt; ++u) {
            if (sdot == 1) acc[NA - 1] += grp_dot(ue[u], ue[u]);
            if (WITH_W && sdot == 2) acc[NA - 1] += grp_dot(ue[u], we[u]);
            if (WITH_W && sdot == 3) acc[NA - 1] += grp_dot(we[u], we[u]);
        }
    };
    int64_t p = lo + lane;
    for (; p + (kDotsU - 1) * 64 < hi; p += kDotsU * 64) {
        Grp<TV> ue[kDotsU], we[kDotsU];
#pragma unroll
        for (int u = 0; u < kDotsU; ++u) {
            ue[u] = ld_grp<AL, false>(um, p + u * 64);
            if (WITH_W) we[u] = ld_grp<AL, false>(wm, p + u * 64);
        }
#pragma unroll
        for (int k = 0; k < NPW; ++k) {
            const int i = wave + 4 * k;
            if (i < nv) {
#pragma unroll
                for (int u = 0; u < kDotsU; ++u) {
                    const Grp<TV> v = ld_grp<AL, true>(Vm + i * vstride, p + u * 64);
                    acc[k] += grp_dot(v, ue[u]);
                    if (WITH_W) acc[NPW + k] += grp_dot(v, we[u]);
                }
            }
        }
        add(ue, we, kDotsU);
    }
    for (; p < hi; p += 64) {
        Grp<TV> ue = ld_grp<AL, false>(um, p), we;
        if (WITH_W) we = ld_grp<AL, false>(wm, p);
#pragma unroll
        for (int k = 0; k < NPW; ++k) {
            const int i = wave + 4 * k;
            if (i < nv) {
                const Grp<TV> v = ld_grp<AL, true>(Vm + i * vstride, p);
                acc[k] += grp_dot(v, ue);
                if (WITH_W) acc[NPW + k] += grp_dot(v, we);
            }
        }
        add(&ue, &we, 1);
    }
    // the n mod GW last elements, by lane 0 of the last block
    if (blockIdx.x == nblk - 1 && lane == 0) {
        for (int64_t e = (n / GW) * GW; e < n; ++e) {
            const double ue = (double)um[e], we = WITH_W ? (double)wm[e] : 0.0;
#pragma unroll
            for (int k = 0; k < NPW; ++k) {
                const int i = wave + 4 * k;
                if (i < nv) {
                    const double v = (double)Vm[i * vstride + e];
                    acc[k] += v * ue;
                    if (WITH_W) acc[NPW + k] += v * we;
                }
            }
            if (sdot == 1) acc[NA - 1] += ue * ue;
            if (WITH_W && sdot == 2) acc[NA - 1] += ue * we;
            if (WITH_W && sdot == 3) acc[NA - 1] += we * we;
        }
    }
    double* pm = partial + (int64_t)mem * kSlots * nblk + blockIdx.x;
#pragma unroll
    for (int k = 0; k < NPW; ++k) {
        const int i = wave + 4 * k;
        if (i < nv) {
            const double a = wave_sum(acc[k]);
            if (lane == 0) pm[(int64_t)i * nblk] = a;
            if (WITH_W) {
                const double t = wave_sum(acc[NPW + k]);
                if (lane == 0) pm[(int64_t)(nv + i) * nblk] = t;
            }
        }
    }
    if (sdot >= 1) {
        const double d = wave_sum(acc[NA - 1]);
        const int slot = WITH_W ? 2 * nv + sdot - 1 : nv;
        if (lane == 0) pm[(int64_t)slot * nblk] = d;
    }
}

// 16-byte group loads need the member's first element and the basis slot
// stride to be multiples of the group (allocations are 256-byte aligned).
template <typename TV>
__device__ __forceinline__ bool groups_aligned(int64_t vstride, int64_t mstride) {
    constexpr int GW = Grp<TV>::GW;
    return ((blockIdx.y * mstride) % GW) == 0 && (vstride % GW) == 0;
}

template <int NPW, bool WITH_W, typename TV>
__global__ __launch_bounds__(RB) void k_dcgs_dots(const TV* __restrict__ V, int64_t vstride, int nv,
                                                  const TV* __restrict__ w, int64_t n, int64_t mstride,
                                                  const int* __restrict__ active, const int* __restrict__ pending,
                                                  double* __restrict__ partial, int nblk) {
    const int mem = blockIdx.y;
    if (!active[mem] && !pending[mem]) return;
    if (groups_aligned<TV>(vstride, mstride))
        dcgs_dots_body<NPW, WITH_W, true>(V, vstride, nv, w, n, mstride, partial, nblk);
    else
        dcgs_dots_body<NPW, WITH_W, false>(V, vstride, nv, w, n, mstride, partial, nblk);
}

// Update pass: basis slot nv+1 = (w - sum_{i<=nv} s_i U_i) / nu with
// s_i = coef[mem*kSlots + i] and 1/nu = scal[mem*4 + 2]; reads slots 0..nv and
// w, writes slot nv+1 only.  NT >= nv + 1 terms; element groups as above.
template <int NT, bool AL, typename TV>
__device__ __forceinline__ void dcgs_update_body(TV* __restrict__ V, int64_t vstride, int nv,
                                                 const TV* __restrict__ w, int64_t n, int64_t mstride,
                                                 const double* sv, double inv_nu, int nblk) {
    constexpr int GW = Grp<TV>::GW;
    const int mem = blockIdx.y;
    const TV* Vm = V + mem * mstride;
    TV* un = V + mem * mstride + (nv + 1) * vstride;
    const TV* wm = w + mem * mstride;
    // Trips of kUpdU * RB element groups are dealt to the blocks in turn (trip
    // t to block t mod nblk), so the blocks in flight stream one contiguous
    // window of every basis vector rather than nblk separate chunks of each
    // (far fewer pages in use at once on large vectors).  No reduction here:
    // each element's arithmetic is the same whatever block computes it.
    const int64_t ngrp = n / GW;
    constexpr int64_t TRIP = (int64_t)kUpdU * RB;
    int64_t base = (int64_t)blockIdx.x * TRIP;
    for (; base + TRIP <= ngrp; base += (int64_t)nblk * TRIP) {
        const int64_t p = base + threadIdx.x;
        Grp<TV> acc[kUpdU];
#pragma unroll
        for (int u = 0; u < kUpdU; ++u) acc[u] = ld_grp<AL, true>(wm, p + u * RB);
#pragma unroll
        for (int i = 0; i < NT; ++i) {
            if (i <= nv) {
#pragma unroll
                for (int u = 0; u < kUpdU; ++u) {
                    const Grp<TV> v = ld_grp<AL, true>(Vm + i * vstride, p + u * RB);
#pragma unroll
                    for (int e = 0; e < GW; ++e) acc[u].v[e] -= sv[i] * v.v[e];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kUpdU; ++u) {
#pragma unroll
            for (int e = 0; e < GW; ++e) acc[u].v[e] *= inv_nu;
            st_grp<AL>(un, p + u * RB, acc[u]);
        }
    }
    // the partial last trip, if any, falls to exactly one block
    for (int64_t p = base + threadIdx.x; p < ngrp; p += RB) {
        Grp<TV> acc = ld_grp<AL, true>(wm, p);
#pragma unroll
        for (int i = 0; i < NT; ++i) {
            if (i <= nv) {
                const Grp<TV> v = ld_grp<AL, true>(Vm + i * vstride, p);
#pragma unroll
                for (int e = 0; e < GW; ++e) acc.v[e] -= sv[i] * v.v[e];
            }
        }
#pragma unroll
        for (int e = 0; e < GW; ++e) acc.v[e] *= inv_nu;
        st_grp<AL>(un, p, acc);
    }
    if (blockIdx.x == nblk - 1 && threadIdx.x == 0) {   // the n mod GW last elements
        for (int64_t e = ngrp * GW; e < n; ++e) {
            double acc = (double)wm[e];
            for (int i = 0; i <= nv; ++i) acc -= sv[i] * (double)Vm[i * vstride + e];
            un[e] = (TV)(acc * inv_nu);
        }
    }
}

template <int NT, typename TV>
__global__ __launch_bounds__(RB) void k_dcgs_update(TV* __restrict__ V, int64_t vstride, int nv,
                                                    const TV* __restrict__ w, int64_t n, int64_t mstride,
                                                    const double* __restrict__ coef, const double* __restrict__ scal,
                                                    const int* __restrict__ active, int nblk) {
    const int mem = blockIdx.y;
    if (!active[mem]) return;                       // uniform per block, before the barrier
    __shared__ double sv[NT];                       // broadcast reads; keeps the lanes' registers for loads
    if ((int)threadIdx.x < NT) sv[threadIdx.x] = (int)threadIdx.x <= nv ? coef[mem * kSlots + threadIdx.x] : 0.0;
    __syncthreads();
    const double inv_nu = scal[mem * 4 + 2];
    if (groups_aligned<TV>(vstride, mstride))
        dcgs_update_body<NT, true>(V, vstride, nv, w, n, mstride, sv, inv_nu, nblk);
    else
        dcgs_update_body<NT, false>(V, vstride, nv, w, n, mstride, sv, inv_nu, nblk);
}

// out[mem*out_stride + out_offset + i] = sum_blk partial[(mem*kSlots + i)*nblk + blk]
__global__ __launch_bounds__(RB) void k_reduce_partials(const double* __restrict__ partial, int nblk, int nv,
                                                        double* __restrict__ out, int out_stride, int out_offset) {
    const int i = blockIdx.x, mem = blockIdx.y;
    __shared__ double red[RB];
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += RB) s += partial[((int64_t)mem * kSlots + i) * nblk + b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = RB / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[mem * out_stride + out_offset + i] = red[0];
}

__global__ void k_scale_vec(double* v, const double* sdev, int sstride, int64_t n, int64_t mstride) {
    const int mem = blockIdx.y;
    const double s = sdev[mem * sstride];
    double* vm = v + mem * mstride;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        vm[e] *= s;
}

template <typename TD>
__global__ void k_copy_scale(const double* src, TD* dst, const double* s, int64_t n, int64_t mstride) {
    const int mem = blockIdx.y;
    const double f = s[mem];
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        dst[mem * mstride + e] = (TD)(f * src[mem * mstride + e]);
}

// x += sum_{i < nv_mem[mem]} y_i Z_i
template <typename TZ>
__global__ void k_multi_axpy(const TZ* __restrict__ Z, int64_t zstride, int nv_max, const int* __restrict__ nv_mem,
                             const double* __restrict__ y, int ystride, double* __restrict__ x, int64_t n,
                             int64_t mstride) {
    const int mem = blockIdx.y;
    const int nv = nv_mem[mem];
    if (nv <= 0) return;
    const double* ym = y + mem * ystride;
    double* xm = x + mem * mstride;
    const TZ* Zm = Z + mem * mstride;
    const int nvv = nv < nv_max ? nv : nv_max;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        double s = xm[e];
        // loads eight vectors ahead of the (in-order) accumulation
        int i = 0;
        for (; i + 8 <= nvv; i += 8) {
            double z[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) z[u] = (double)Zm[(int64_t)(i + u) * zstride + e];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += ym[i + u] * z[u];
        }
        for (; i < nvv; ++i) s += ym[i] * (double)Zm[(int64_t)i * zstride + e];
        xm[e] = s;
    }
}

// r = b - r; partial ||r||^2
__global__ __launch_bounds__(RB) void k_sub_norm(const double* __restrict__ b, double* __restrict__ r, int64_t n,
                                                 int64_t mstride, double* __restrict__ partial, int nblk) {
    const int mem = blockIdx.y;
    int64_t lo, hi;
    chunk_range(n, nblk, blockIdx.x, lo, hi);
    double acc[1] = {0.0};
    for (int64_t e = lo + threadIdx.x; e < hi; e += RB) {
        const double v = b[mem * mstride + e] - r[mem * mstride + e];
        r[mem * mstride + e] = v;
        acc[0] += v * v;
    }
    block_reduce_store<1>(acc, 1, partial, mem, kSlots, nblk);
}

__global__ __launch_bounds__(RB) void k_norm(const double* __restrict__ x, int64_t n, int64_t mstride,
                                             double* __restrict__ partial, int nblk) {
    const int mem = blockIdx.y;
    int64_t lo, hi;
    chunk_range(n, nblk, blockIdx.x, lo, hi);
    double acc[1] = {0.0};
    for (int64_t e = lo + threadIdx.x; e < hi; e += RB) {
        const double v = x[mem * mstride + e];
        acc[0] += v * v;
    }
    block_reduce_store<1>(acc, 1, partial, mem, kSlots, nblk);
}

__global__ void k_axpby(double a, const double* x, double b, double* y, int64_t n) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        y[e] = a * x[e] + b * y[e];
}

__global__ void k_cast_d2f(const double* x, float* y, int64_t n) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        y[e] = (float)x[e];
}
__global__ void k_cast_f2d(const float* x, double* y, int64_t n) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        y[e] = (double)x[e];
}

// Arnoldi column j: H(0..j, j) = h1 + h2, H(j+1, j) = ||w2||; previous Givens
// rotations, new rotation, g update, residual estimate.  nrm holds ||w2||^2 on
// entry and 1/||w2|| (0 at breakdown) on exit.
__global__ void k_arnoldi_finish(KrylovDev k, int restart, int j, int nmem) {
    const int mem = blockIdx.x * blockDim.x + threadIdx.x;
    if (mem >= nmem) return;
    if (!k.active[mem]) return;
    const int ld = restart + 1;
    double* H = k.H + (int64_t)mem * ld * restart;
    double* col = H + (int64_t)j * ld;
    const double* h1 = k.h1 + mem * ld;
    const double* h2 = k.h2 + mem * ld;
    for (int i = 0; i <= j; ++i) col[i] = h1[i] + h2[i];
    const double nn = sqrt(k.nrm[mem]);
    col[j + 1] = nn;
    k.nrm[mem] = nn > 0.0 ? 1.0 / nn : 0.0;
    double* cs = k.cs + mem * restart;
    double* sn = k.sn + mem * restart;
    for (int i = 0; i < j; ++i) {
        const double a = col[i], b = col[i + 1];
        col[i] = cs[i] * a + sn[i] * b;
        col[i + 1] = -sn[i] * a + cs[i] * b;
    }
    const double a = col[j], b = col[j + 1];
    const double den = hypot(a, b);
    const double c = den > 0.0 ? a / den : 1.0;
    const double s = den > 0.0 ? b / den : 0.0;
    cs[j] = c;
    sn[j] = s;
    col[j] = den;
    col[j + 1] = 0.0;
    double* g = k.g + mem * ld;
    g[j + 1] = -s * g[j];
    g[j] = c * g[j];
    k.resid[mem] = fabs(g[j + 1]);
}

// Givens rotations 0..j-1 applied to a column, rotation j formed from (col[j], col[j+1]).
__device__ void givens_column(double* col, double* cs, double* sn, double* g, int j) {
    for (int i = 0; i < j; ++i) {
        const double a = col[i], b = col[i + 1];
        col[i] = cs[i] * a + sn[i] * b;
        col[i + 1] = -sn[i] * a + cs[i] * b;
    }
    const double a = col[j], b = col[j + 1];
    const double den = hypot(a, b);
    const double c = den > 0.0 ? a / den : 1.0;
    const double s = den > 0.0 ? b / den : 0.0;
    cs[j] = c;
    sn[j] = s;
    col[j] = den;
    col[j + 1] = 0.0;
    g[j + 1] = -s * g[j];
    g[j] = c * g[j];
}

// DCGS2 bookkeeping of iteration j (mode 0) or of the last column (mode 1).
// The basis slots keep the candidates U_i (never rewritten); the orthonormal
// basis is V = U R^{-1} with R upper triangular (R column i = [a; rho] from
// U_i = sum_l a_l V_l + rho V_i), so dots against U become dots against V by a
// triangular solve.  Commit: the candidate u_j of the previous iteration gives
// a = V_{<j}^T u_j, rho^2 = u.u - |a|^2, and column j-1 (raw entries t, c, nu)
// becomes [t + nu a, c + nu a_{j-1}, nu rho] and gets its Givens rotation.
// Provisional (mode 0, active members): column j = [t, c, nu] with t = V^T w,
// c = (u.w - a.t) / rho and nu^2 = w.w - |t|^2 - c^2 (one Gram-Schmidt pass);
// its rotation on a copy gives the residual estimate used to stop.  The
// update pass then needs s = R^{-1} [t; c]: u_{j+1} = (w - sum_{i<=j} s_i U_i) / nu.
// One 64-thread block per member: the block stages the member's R (the
// (j+1) x (j+1) leading part), reduced dots, rotations, right-hand side and the
// two Hessenberg columns in LDS, lane 0 runs the O(j^2) recurrences there (no
// dependent global loads) and the block writes the touched entries back.
__global__ __launch_bounds__(64) void k_dcgs_finish(KrylovDev k, int restart, int j, int mode, int nmem) {
    constexpr int LR = 32;                         // LDS leading dimension (restart <= 31)
    const int mem = blockIdx.x;
    const int tid = threadIdx.x;
    const int ld = restart + 1;
    const int nv = j;
    __shared__ double sR[LR * LR];                 // R(l, i) at [l + LR i], l, i <= j
    __shared__ double sD[kSlots];
    __shared__ double scs[LR], ssn[LR], sg[LR + 1];
    __shared__ double sc0[LR + 1], sc1[LR + 1];    // Hessenberg columns j-1 and j
    __shared__ double ssv[LR];                     // update coefficients s
    __shared__ double a[LR], t[LR];                // V^T u_j and V^T w
    __shared__ int flags[2];                       // [0]: committed column j-1, [1]: provisional column j
    const double* D = k.dots + (int64_t)mem * kSlots;
    double* H = k.H + (int64_t)mem * ld * restart;
    double* R = k.R + (int64_t)mem * ld * ld;      // R[l + i*ld] = R(l, i)
    double* cs = k.cs + mem * restart;
    double* sn = k.sn + mem * restart;
    double* g = k.g + mem * ld;
    double* sc = k.scal + mem * 4;
    for (int q = tid; q < (j + 1) * (j + 1); q += 64) {
        const int l = q % (j + 1), i = q / (j + 1);
        sR[l + LR * i] = R[l + i * ld];
    }
    for (int q = tid; q < kSlots; q += 64) sD[q] = D[q];
    for (int q = tid; q < j; q += 64) {
        scs[q] = cs[q];
        ssn[q] = sn[q];
    }
    for (int q = tid; q <= j + 1 && q < ld; q += 64) sg[q] = g[q];
    if (j >= 1)
        for (int q = tid; q <= j; q += 64) sc0[q] = H[(int64_t)(j - 1) * ld + q];
    __syncthreads();
    if (tid == 0) {
        // out = R_{<j}^{-T} d (forward substitution)
        auto lower_solve = [&](const double* d, double* out) {
            for (int l = 0; l < nv; ++l) {
                double v = d[l];
                for (int p = 0; p < l; ++p) v -= sR[p + l * LR] * out[p];
                const double dl = sR[l + l * LR];
                out[l] = dl != 0.0 ? v / dl : 0.0;
            }
        };
        for (int i = 0; i < LR; ++i) a[i] = t[i] = 0.0;
        flags[0] = flags[1] = 0;
        double rho = 1.0;                          // R(0, 0) = 1: U_0 = V_0
        if (j >= 1 && k.pending[mem]) {
            lower_solve(sD, a);
            const double alpha = mode ? sD[nv] : sD[2 * nv];
            double a2 = 0.0;
            for (int i = 0; i < nv; ++i) a2 += a[i] * a[i];
            rho = sqrt(fmax(alpha - a2, 0.0));
            for (int l = 0; l < nv; ++l) sR[l + j * LR] = a[l];
            sR[j + j * LR] = rho;
            const double nu = sc[3];
            for (int i = 0; i < nv; ++i) sc0[i] += nu * a[i];
            sc0[j] = nu * rho;
            givens_column(sc0, scs, ssn, sg, j - 1);
            k.resid[mem] = fabs(sg[j]);
            k.pending[mem] = 0;
            flags[0] = 1;
        }
        if (mode == 0 && k.active[mem]) {
            lower_solve(sD + nv, t);
            double at = 0.0, t2 = 0.0;
            for (int i = 0; i < nv; ++i) {
                at += a[i] * t[i];
                t2 += t[i] * t[i];
            }
            const double c = rho > 0.0 ? (sD[2 * nv + 1] - at) / rho : 0.0;
            const double nu = sqrt(fmax(sD[2 * nv + 2] - t2 - c * c, 0.0));
            for (int i = 0; i < nv; ++i) sc1[i] = t[i];
            sc1[j] = c;
            sc1[j + 1] = nu;
            // provisional rotation: entry j of the column after rotations 0..j-1
            double xr = sc1[0];
            for (int i = 0; i < j; ++i) xr = -ssn[i] * xr + scs[i] * sc1[i + 1];
            const double den = hypot(xr, nu);
            k.resid[mem] = den > 0.0 ? fabs(nu / den * sg[j]) : 0.0;
            // s = R_{<=j}^{-1} [t; c] (back substitution)
            for (int l = j; l >= 0; --l) {
                double v = l == j ? c : t[l];
                for (int p = l + 1; p <= j; ++p) v -= sR[l + p * LR] * ssv[p];
                const double dl = sR[l + l * LR];
                ssv[l] = dl != 0.0 ? v / dl : 0.0;
            }
            sc[2] = nu > 0.0 ? 1.0 / nu : 0.0;
            sc[3] = nu;
            k.pending[mem] = 1;
            flags[1] = 1;
        }
    }
    __syncthreads();
    if (flags[0]) {
        for (int q = tid; q <= j; q += 64) {
            R[q + j * ld] = sR[q + j * LR];
            H[(int64_t)(j - 1) * ld + q] = sc0[q];
        }
        if (tid == 0) {
            cs[j - 1] = scs[j - 1];
            sn[j - 1] = ssn[j - 1];
            g[j - 1] = sg[j - 1];
            g[j] = sg[j];
        }
    }
    if (flags[1]) {
        for (int q = tid; q <= j + 1; q += 64) H[(int64_t)j * ld + q] = sc1[q];
        double* sv = k.coef + (int64_t)mem * kSlots;
        for (int q = tid; q <= j; q += 64) sv[q] = ssv[q];
    }
}

__global__ void k_cycle_start(KrylovDev k, int restart, const double* beta0sq, int nmem) {
    const int mem = blockIdx.x * blockDim.x + threadIdx.x;
    if (mem >= nmem) return;
    const int ld = restart + 1;
    double* g = k.g + mem * ld;
    for (int i = 0; i < ld; ++i) g[i] = 0.0;
    const double b = sqrt(beta0sq[mem]);
    g[0] = b;
    k.nrm[mem] = b > 0.0 ? 1.0 / b : 0.0;
    k.resid[mem] = b;
    k.pending[mem] = 0;
    k.scal[mem * 4 + 3] = 1.0;     // V_0 = r / ||r|| is final as written
    k.R[(int64_t)mem * ld * ld] = 1.0;
}

// y = R^{-1} g on the leading jend x jend block (upper triangular after Givens).
__global__ void k_back_solve(KrylovDev k, int restart, const int* jend, int nmem) {
    const int mem = blockIdx.x * blockDim.x + threadIdx.x;
    if (mem >= nmem) return;
    const int ld = restart + 1;
    const int m = jend[mem];
    const double* H = k.H + (int64_t)mem * ld * restart;
    const double* g = k.g + mem * ld;
    double* y = k.y + mem * restart;
    for (int i = m - 1; i >= 0; --i) {
        double s = g[i];
        for (int q = i + 1; q < m; ++q) s -= H[i + (int64_t)q * ld] * y[q];
        const double d = H[i + (int64_t)i * ld];
        y[i] = d != 0.0 ? s / d : 0.0;
    }
}

// Richardson residual on field columns: out = R - off_scale Y - b1 M V (the
// mean block's mass part and the off-level SG products Y = SG_r(V) of
// Z_r = I (x) (a1 K + b1 M) + off_scale sum_k G_k (x) K_k, whose a1 K part Y
// also carries); member of column c = c / cpv (0 when shared).
template <typename T>
__global__ void k_z_residual(int n, const T* __restrict__ R, ColMap rmap, const T* __restrict__ Y,
                             const T* __restrict__ V, ColMap vmap, T* __restrict__ out, ColMap omap,
                             const MemberDev* __restrict__ mem, int cpv, int shared, const int* __restrict__ act) {
    const int c = blockIdx.y;
    const int vec = c / cpv;
    if (act && !act[vec]) return;
    const int N1 = n + 1;
    const int64_t nodes = (int64_t)N1 * N1;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nodes) return;
    const int ix = (int)(q % N1), iy = (int)(q / N1);
    T* o = out + omap.off(c);
    if (ix == 0 || iy == 0 || ix == n || iy == n) {
        o[q] = T(0);
        return;
    }
    const MemberDev md = mem[shared ? 0 : vec];
    const T* v = V + vmap.off(c);
    const double h = 1.0 / n;
    const double w = h * h / 36.0;
    const double m9 = w * (16.0 * (double)v[q] +
                           4.0 * ((double)v[q - 1] + (double)v[q + 1] + (double)v[q - N1] + (double)v[q + N1]) +
                           ((double)v[q - N1 - 1] + (double)v[q - N1 + 1] + (double)v[q + N1 - 1] +
                            (double)v[q + N1 + 1]));
    const double y = (double)Y[vmap.off(c) + q];
    o[q] = (T)((double)R[rmap.off(c) + q] - md.off_scale * y - md.b1 * m9);
}

// out = A + B column by column (every node)
template <typename T>
__global__ void k_cols_add(int64_t nodes, const T* __restrict__ A, ColMap amap, const T* __restrict__ Bv, ColMap bmap,
                           T* __restrict__ out, ColMap omap, int cpv, const int* __restrict__ act) {
    const int c = blockIdx.y;
    if (act && !act[c / cpv]) return;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nodes) return;
    out[omap.off(c) + q] = A[amap.off(c) + q] + Bv[bmap.off(c) + q];
}

__global__ void k_conv_check(KrylovDev k, int j, int nmem) {
    const int mem = blockIdx.x * blockDim.x + threadIdx.x;
    if (mem >= nmem || !k.active[mem]) return;
    k.jend[mem] = j + 1;
    const int it = k.iters[mem] + 1;
    k.iters[mem] = it;
    if (k.resid[mem] <= k.tol[mem] || it >= k.itmax[mem]) k.active[mem] = 0;
}

int grid1d(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return (int)b;
}

dim3 tile_grid(int n, int nchunks, int64_t slices) {
    const int tiles = ((n + 1 + TX - 1) / TX) * ((n + 1 + TY - 1) / TY);
    if (slices > 65535 || nchunks > 65535) throw Error(SG_ERR_INVALID, "launch grid too large");
    return dim3(tiles, nchunks, (unsigned)slices);
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T>
void launch_sg_apply(const Shape& s, const OpDev& op, const T* x, T* y, int nvec, uint32_t mask, hipStream_t st) {
    if (op.gen) {
        // general coupling: all terms, or (mask below all ones) the terms l < r of genBr
        const ColMap full = [&] {
            ColMap m;
            m.mstride = s.blk;
            m.tstride = s.tstride;
            m.nodes = s.nodes;
            m.L = s.nxi;
            m.nt = s.nt;
            m.j0 = 0;
            return m;
        }();
        launch_gen_sg<T>(s, op, mask != 0xffffffffu, x, s.blk, s.tstride, 0, s.nxi, 0, 0, 0, s.nxi, (const T*)nullptr,
                         full, y, full, 1.0, 0, 0.0, nvec, st);
        return;
    }
    if (launch_sgx_apply<T>(s, op, x, y, nvec, mask, st)) return;
    dim3 g = tile_grid(s.n, (s.nxi + kJChunk - 1) / kJChunk, (int64_t)nvec * s.nt);
    hipLaunchKernelGGL(k_sg_apply<T>, g, dim3(256), 0, st, s.n, s.M, s.nxi, s.nt, s.nodes, op, x, y, mask);
    SG_HIP(hipGetLastError());
}

template <typename T>
void launch_kkt_apply(const Shape& s, const OpDev& op, const T* x, T* y, int nvec, hipStream_t st) {
    if (op.gen) throw Error(SG_ERR_INVALID, "internal: the general-coupling KKT apply needs scratch (launch_gen_kkt)");
    if (launch_sgx_kkt<T>(s, op, x, y, nvec, st)) return;
    dim3 g = tile_grid(s.n, (s.nxi + kJChunk - 1) / kJChunk, (int64_t)nvec * s.nt);
    hipLaunchKernelGGL(k_kkt_apply<T>, g, dim3(256), 0, st, s.n, s.M, s.nxi, s.nt, (int)s.time, s.nodes, op, x, y);
    SG_HIP(hipGetLastError());
}

template <typename T>
void launch_hgs_rhs(const Shape& s, const OpDev& op, int d, uint32_t mask, int use_lower, int use_upper,
                    const T* base, ColMap bmap, const T* V, ColMap vmap, T* out, ColMap omap, int nmembers,
                    hipStream_t st) {
    if (op.gen) {
        // the coupled columns of every other level: all lower ones and/or all upper ones;
        // base - off_sign * off_scale (couplings) with the member's off_scale
        const int lo = s.off[d], hi = s.off[d + 1];
        launch_gen_sg<T>(s, op, true, V, vmap.mstride, vmap.tstride, 0, use_lower ? lo : 0, hi,
                         use_upper ? s.nxi : hi, lo, hi - lo, base, bmap, out, omap, 0.0, op.off_sign > 0 ? 1 : -1,
                         0.0, nmembers, st);
        return;
    }
    if (launch_sgx_hgs_rhs<T>(s, op, d, mask, use_lower, use_upper, base, bmap, V, vmap, out, omap, nmembers, st))
        return;
    const int L = s.off[d + 1] - s.off[d];
    dim3 g = tile_grid(s.n, (L + kJChunk - 1) / kJChunk, (int64_t)nmembers * s.nt);
    hipLaunchKernelGGL(k_hgs_rhs<T>, g, dim3(256), 0, st, s.n, s.M, s.nxi, s.nt, s.nodes, op, s.off[d], L, mask,
                       use_lower, use_upper, base, bmap, V, vmap, out, omap);
    SG_HIP(hipGetLastError());
}

template <typename T>
void launch_mass_cheb(const Shape& s, const OpDev& op, const T* r, T* z, T* bufA, T* bufB, int nvec, int steps,
                      hipStream_t st) {
    if (launch_mass_cheb_fused<T>(s, op, r, z, nvec, steps, st)) return;
    const int ncols = 2 * s.nt * s.nxi;
    dim3 g = tile_grid(s.n, (ncols + kJChunk - 1) / kJChunk, nvec);
    const int64_t vstride = 3 * s.blk;
    const double rho = 0.8;
    // x_1 = D^{-1} r (omega_1 = 1); buffers: prev = A, cur = B
    T* prev = bufA;
    T* cur = bufB;
    hipLaunchKernelGGL(k_mass_cheb_step<T>, g, dim3(256), 0, st, s.n, s.nxi, s.nt, (int)s.time, s.nodes, op, vstride,
                       r, (const T*)nullptr, (const T*)nullptr, steps == 1 ? z : cur, T(1), 1, steps == 1 ? 1 : 0);
    SG_HIP(hipGetLastError());
    if (steps == 1) return;
    // prev holds x_0 = 0 (a fill kernel, not a memset node, so that the
    // sequence can be captured in a graph)
    const int64_t cnt = (int64_t)nvec * ncols * s.nodes;
    hipLaunchKernelGGL(k_fill_zero<T>, dim3(grid1d(cnt)), dim3(256), 0, st, prev, cnt);
    SG_HIP(hipGetLastError());
    double omega = 1.0;
    for (int k = 1; k < steps; ++k) {
        omega = (k == 1) ? 1.0 / (1.0 - 0.5 * rho * rho) : 1.0 / (1.0 - 0.25 * rho * rho * omega);
        const bool last = (k == steps - 1);
        T* out = last ? z : prev;   // x_{k+1} overwrites x_{k-1}
        hipLaunchKernelGGL(k_mass_cheb_step<T>, g, dim3(256), 0, st, s.n, s.nxi, s.nt, (int)s.time, s.nodes, op,
                           vstride, r, (const T*)cur, (const T*)prev, out, T(omega), 0, last ? 1 : 0);
        SG_HIP(hipGetLastError());
        if (!last) std::swap(prev, cur);
    }
}

template <typename T>
void launch_mass_scaled(const Shape& s, const OpDev& op, const T* V, ColMap vmap, T* W, ColMap wmap, int ncols,
                        int, hipStream_t st) {
    const int tiles_x = (s.n + 1 + 29) / 30, tiles_y = (s.n + 1 + 2 * kMassRows - 1) / (2 * kMassRows);
    const int chunks = (ncols + 3) / 4;
    if (chunks > 65535) throw Error(SG_ERR_INVALID, "mass apply: too many columns in one launch");
    hipLaunchKernelGGL(k_mass_scaled<T>, dim3(tiles_x * tiles_y, chunks), dim3(256), 0, st, s.n, s.nt, (int)s.time,
                       op, V, vmap, W, wmap, ncols, tiles_x);
    SG_HIP(hipGetLastError());
}






template <>
void launch_mg_coarse<double>(const double* ainv, const double* bc, ColMap bmap, double* xc, ColMap xmap, int ncols,
                              int cpm, hipStream_t st) {
    const int nmem = (ncols + cpm - 1) / cpm;
    dim3 g((cpm + 15) / 16, nmem);
    hipLaunchKernelGGL(k_mg_coarse_f64, g, dim3(64), 0, st, ainv, bc, bmap, xc, xmap, ncols, cpm);
    SG_HIP(hipGetLastError());
}

template <>
void launch_mg_coarse<float>(const float* ainv, const float* bc, ColMap bmap, float* xc, ColMap xmap, int ncols,
                             int cpm, hipStream_t st) {
    const int nmem = (ncols + cpm - 1) / cpm;
    dim3 g(cpm, nmem);
    hipLaunchKernelGGL(k_mg_coarse_f32, g, dim3(64), 0, st, ainv, bc, bmap, xc, xmap, ncols, cpm);
    SG_HIP(hipGetLastError());
}

template <typename T>
void launch_fill_zero(T* x, int64_t count, hipStream_t st) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_fill_zero<T>, dim3(grid1d(count)), dim3(256), 0, st, x, count);
    SG_HIP(hipGetLastError());
}
template void launch_fill_zero<double>(double*, int64_t, hipStream_t);
template void launch_fill_zero<float>(float*, int64_t, hipStream_t);

template <typename T>
void launch_zero_ring(T* x, int n, int64_t ncols, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_ring<T>, dim3(grid1d(4 * (int64_t)n * ncols)), dim3(256), 0, st, x, n, ncols);
    SG_HIP(hipGetLastError());
}

// Instantiations by basis-vector count: fewer accumulators for short bases.
#define SG_NV_DISPATCH(KERNEL, nv, ...)                                                          \
    do {                                                                                          \
        if ((nv) <= 4)                                                                            \
            hipLaunchKernelGGL(KERNEL<4>, __VA_ARGS__);                                           \
        else if ((nv) <= 8)                                                                       \
            hipLaunchKernelGGL(KERNEL<8>, __VA_ARGS__);                                           \
        else if ((nv) <= 16)                                                                      \
            hipLaunchKernelGGL(KERNEL<16>, __VA_ARGS__);                                          \
        else                                                                                      \
            hipLaunchKernelGGL(KERNEL<32>, __VA_ARGS__);                                          \
    } while (0)

void launch_multidot(const double* V, int64_t vstride, int nv, const double* w, int64_t n, int nmem, int64_t mstride,
                     double* partial, int nblk, hipStream_t st) {
    if (nv > MAXV) throw Error(SG_ERR_INVALID, "multidot: too many vectors");
    SG_NV_DISPATCH(k_multidot, nv, dim3(nblk, nmem), dim3(RB), 0, st, V, vstride, nv, w, n, mstride, partial, nblk);
    SG_HIP(hipGetLastError());
}

void launch_cgs_update_dot(const double* V, int64_t vstride, int nv, const double* h, int hstride, double* w,
                           int64_t n, int nmem, int64_t mstride, double* partial, int nblk, hipStream_t st) {
    if (nv > MAXV) throw Error(SG_ERR_INVALID, "cgs: too many vectors");
    SG_NV_DISPATCH(k_cgs_update_dot, nv, dim3(nblk, nmem), dim3(RB), 0, st, V, vstride, nv, h, hstride, w, n,
                   mstride, partial, nblk);
    SG_HIP(hipGetLastError());
}

void launch_cgs_update_norm(const double* V, int64_t vstride, int nv, const double* h, int hstride, const double* w,
                            double* out, int64_t n, int nmem, int64_t mstride, double* partial, int nblk,
                            hipStream_t st) {
    if (nv > MAXV) throw Error(SG_ERR_INVALID, "cgs: too many vectors");
    SG_NV_DISPATCH(k_cgs_update_norm, nv, dim3(nblk, nmem), dim3(RB), 0, st, V, vstride, nv, h, hstride, w, out, n,
                   mstride, partial, nblk);
    SG_HIP(hipGetLastError());
}

template <typename TV>
void launch_dcgs_dots(const TV* V, int64_t vstride, int nv, const TV* w, int64_t n, int nmem, int64_t mstride,
                      const int* active, const int* pending, double* partial, int nblk, hipStream_t st) {
    if (nv > (w ? MAXV - 2 : MAXV)) throw Error(SG_ERR_INVALID, "dcgs: too many vectors");
    const dim3 g(nblk, nmem), b(RB);
#define SG_DOTS(NPW, WW)                                                                                            \
    hipLaunchKernelGGL((k_dcgs_dots<NPW, WW, TV>), g, b, 0, st, V, vstride, nv, w, n, mstride, active, pending,     \
                       partial, nblk)
    if (w) {
        if (nv <= 4) SG_DOTS(1, true);
        else if (nv <= 8) SG_DOTS(2, true);
        else if (nv <= 16) SG_DOTS(4, true);
        else SG_DOTS(8, true);
    } else {
        if (nv <= 4) SG_DOTS(1, false);
        else if (nv <= 8) SG_DOTS(2, false);
        else if (nv <= 16) SG_DOTS(4, false);
        else SG_DOTS(8, false);
    }
#undef SG_DOTS
    SG_HIP(hipGetLastError());
}

template <typename TV>
void launch_dcgs_update(TV* V, int64_t vstride, int nv, const TV* w, int64_t n, int nmem, int64_t mstride,
                        const double* coef, const double* scal, const int* active, int nblk, hipStream_t st) {
    if (nv > MAXV - 2) throw Error(SG_ERR_INVALID, "dcgs: too many vectors");
    const dim3 g(nblk, nmem), b(RB);
    const int nt = nv + 1;
#define SG_UPD(NT) hipLaunchKernelGGL((k_dcgs_update<NT, TV>), g, b, 0, st, V, vstride, nv, w, n, mstride, coef, scal, \
                                      active, nblk)
    if (nt <= 4) SG_UPD(4);
    else if (nt <= 8) SG_UPD(8);
    else if (nt <= 16) SG_UPD(16);
    else SG_UPD(32);
#undef SG_UPD
    SG_HIP(hipGetLastError());
}
template void launch_dcgs_dots<double>(const double*, int64_t, int, const double*, int64_t, int, int64_t, const int*,
                                       const int*, double*, int, hipStream_t);
template void launch_dcgs_dots<float>(const float*, int64_t, int, const float*, int64_t, int, int64_t, const int*,
                                      const int*, double*, int, hipStream_t);
template void launch_dcgs_update<double>(double*, int64_t, int, const double*, int64_t, int, int64_t, const double*,
                                         const double*, const int*, int, hipStream_t);
template void launch_dcgs_update<float>(float*, int64_t, int, const float*, int64_t, int, int64_t, const double*,
                                        const double*, const int*, int, hipStream_t);

void launch_dcgs_finish(KrylovDev k, int restart, int j, int mode, int nmem, hipStream_t st) {
    if (restart > 31) throw Error(SG_ERR_INVALID, "dcgs: restart above 31");
    hipLaunchKernelGGL(k_dcgs_finish, dim3(nmem), dim3(64), 0, st, k, restart, j, mode, nmem);
    SG_HIP(hipGetLastError());
}

void launch_reduce_partials(const double* partial, int nblk, int nv, int nmem, double* out, int out_stride,
                            int out_offset, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_partials, dim3(nv, nmem), dim3(RB), 0, st, partial, nblk, nv, out, out_stride,
                       out_offset);
    SG_HIP(hipGetLastError());
}

void launch_scale_vec(double* v, const double* sdev, int sstride, int64_t n, int nmem, int64_t mstride,
                      hipStream_t st) {
    hipLaunchKernelGGL(k_scale_vec, dim3(grid1d(n), nmem), dim3(256), 0, st, v, sdev, sstride, n, mstride);
    SG_HIP(hipGetLastError());
}

template <typename TD>
void launch_copy_scale_rows(const double* src, TD* dst, const double* inv_norm, int64_t n, int nmem, int64_t mstride,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_copy_scale<TD>, dim3(grid1d(n), nmem), dim3(256), 0, st, src, dst, inv_norm, n, mstride);
    SG_HIP(hipGetLastError());
}
template void launch_copy_scale_rows<double>(const double*, double*, const double*, int64_t, int, int64_t,
                                             hipStream_t);
template void launch_copy_scale_rows<float>(const double*, float*, const double*, int64_t, int, int64_t, hipStream_t);

void launch_multi_axpy(const void* Z, int zfp32, int64_t zstride, int nv_max, const int* nv_mem, const double* y,
                       int ystride, double* x, int64_t n, int nmem, int64_t mstride, hipStream_t st) {
    if (zfp32)
        hipLaunchKernelGGL(k_multi_axpy<float>, dim3(grid1d(n), nmem), dim3(256), 0, st, (const float*)Z, zstride,
                           nv_max, nv_mem, y, ystride, x, n, mstride);
    else
        hipLaunchKernelGGL(k_multi_axpy<double>, dim3(grid1d(n), nmem), dim3(256), 0, st, (const double*)Z, zstride,
                           nv_max, nv_mem, y, ystride, x, n, mstride);
    SG_HIP(hipGetLastError());
}

void launch_sub_norm(const double* b, double* r, int64_t n, int nmem, int64_t mstride, double* partial, int nblk,
                     hipStream_t st) {
    hipLaunchKernelGGL(k_sub_norm, dim3(nblk, nmem), dim3(RB), 0, st, b, r, n, mstride, partial, nblk);
    SG_HIP(hipGetLastError());
}

void launch_norm(const double* x, int64_t n, int nmem, int64_t mstride, double* partial, int nblk, hipStream_t st) {
    hipLaunchKernelGGL(k_norm, dim3(nblk, nmem), dim3(RB), 0, st, x, n, mstride, partial, nblk);
    SG_HIP(hipGetLastError());
}

void launch_axpby(double a, const double* x, double b, double* y, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_axpby, dim3(grid1d(n)), dim3(256), 0, st, a, x, b, y, n);
    SG_HIP(hipGetLastError());
}

void launch_cast_d2f(const double* x, float* y, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_cast_d2f, dim3(grid1d(n)), dim3(256), 0, st, x, y, n);
    SG_HIP(hipGetLastError());
}

void launch_cast_f2d(const float* x, double* y, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_cast_f2d, dim3(grid1d(n)), dim3(256), 0, st, x, y, n);
    SG_HIP(hipGetLastError());
}

void launch_arnoldi_finish(KrylovDev k, int restart, int j, int nmem, hipStream_t st) {
    hipLaunchKernelGGL(k_arnoldi_finish, dim3((nmem + 63) / 64), dim3(64), 0, st, k, restart, j, nmem);
    SG_HIP(hipGetLastError());
}

void launch_cycle_start(KrylovDev k, int restart, const double* beta0sq, int nmem, hipStream_t st) {
    hipLaunchKernelGGL(k_cycle_start, dim3((nmem + 63) / 64), dim3(64), 0, st, k, restart, beta0sq, nmem);
    SG_HIP(hipGetLastError());
}

void launch_back_solve(KrylovDev k, int restart, const int* jend, int nmem, hipStream_t st) {
    hipLaunchKernelGGL(k_back_solve, dim3((nmem + 63) / 64), dim3(64), 0, st, k, restart, jend, nmem);
    SG_HIP(hipGetLastError());
}

template <typename T>
void launch_z_residual(int n, const T* R, ColMap rmap, const T* Y, const T* V, ColMap vmap, T* out, ColMap omap,
                       const MemberDev* mem, int ncols, int cpv, int shared, const int* act, hipStream_t st) {
    if (ncols < 1) return;
    if (ncols > 65535) throw Error(SG_ERR_INVALID, "Richardson residual: too many columns in one launch");
    const int64_t nodes = (int64_t)(n + 1) * (n + 1);
    hipLaunchKernelGGL(k_z_residual<T>, dim3((unsigned)((nodes + 255) / 256), ncols), dim3(256), 0, st, n, R, rmap, Y,
                       V, vmap, out, omap, mem, cpv, shared, act);
    SG_HIP(hipGetLastError());
}

template <typename T>
void launch_cols_add(int64_t nodes, const T* A, ColMap amap, const T* Bv, ColMap bmap, T* out, ColMap omap, int ncols,
                     int cpv, const int* act, hipStream_t st) {
    if (ncols < 1) return;
    if (ncols > 65535) throw Error(SG_ERR_INVALID, "column add: too many columns in one launch");
    hipLaunchKernelGGL(k_cols_add<T>, dim3((unsigned)((nodes + 255) / 256), ncols), dim3(256), 0, st, nodes, A, amap,
                       Bv, bmap, out, omap, cpv, act);
    SG_HIP(hipGetLastError());
}

void launch_conv_check(KrylovDev k, int j, int nmem, hipStream_t st) {
    hipLaunchKernelGGL(k_conv_check, dim3((nmem + 63) / 64), dim3(64), 0, st, k, j, nmem);
    SG_HIP(hipGetLastError());
}

// explicit instantiations
#define SG_INST(T)                                                                                          \
    template void launch_sg_apply<T>(const Shape&, const OpDev&, const T*, T*, int, uint32_t, hipStream_t); \
    template void launch_kkt_apply<T>(const Shape&, const OpDev&, const T*, T*, int, hipStream_t);          \
    template void launch_hgs_rhs<T>(const Shape&, const OpDev&, int, uint32_t, int, int, const T*, ColMap,  \
                                    const T*, ColMap, T*, ColMap, int, hipStream_t);                        \
    template void launch_mass_cheb<T>(const Shape&, const OpDev&, const T*, T*, T*, T*, int, int,           \
                                      hipStream_t);                                                         \
    template void launch_mass_scaled<T>(const Shape&, const OpDev&, const T*, ColMap, T*, ColMap, int, int, \
                                        hipStream_t);                                                       \
    template void launch_zero_ring<T>(T*, int, int64_t, hipStream_t);                                      \
    template void launch_z_residual<T>(int, const T*, ColMap, const T*, const T*, ColMap, T*, ColMap,        \
                                       const MemberDev*, int, int, int, const int*, hipStream_t);           \
    template void launch_cols_add<T>(int64_t, const T*, ColMap, const T*, ColMap, T*, ColMap, int, int,    \
                                     const int*, hipStream_t);
SG_INST(double)
SG_INST(float)

}  // namespace sg
