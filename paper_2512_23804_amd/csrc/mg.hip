// Fused geometric-multigrid kernels for A = a1 K + b1 M_h on one grid level.
//
// One V-cycle level is two launches instead of one per smoothing step:
//   down: x = pre-smoothing of b from a zero guess (NU Chebyshev steps),
//         r = b - A x, b_coarse = P^T r           (b read once, x and b_coarse written)
//   up:   x' = x + P e_coarse, then NU post-smoothing steps from x'
//         (b and x read, x' written)
// Each workgroup stages a tile of the level plus a halo of NU+1 nodes in LDS
// and runs all steps there (the halo shrinks by one node per stencil step),
// so the finest level is read about three times and written about twice
// per V-cycle.  The smoother is the Chebyshev iteration
//   r = b - A x;  d = c_d d + c_r D^{-1} r;  x = x + d
// with per-member, per-level coefficients (c_d = 0 in the first step).
// Tiles start at node 1 (the Dirichlet ring is zero), so 2^k - 1 interior
// nodes per side take 2^k / tile tiles; the first tile row and column also
// write the zero ring at index 0.
#include "common.hpp"

namespace sg {

namespace {

// Column skip of the multigrid kernels: column c is skipped when act != null
// and act[c / cpv] == 0 (cpv: columns per vector).
struct Skip {
    const int* act;
    int cpv;
};


template <typename T>
__device__ __forceinline__ T st9(const T* s, int W, int i, T wc, T we, T wd) {
    return wc * s[i] + we * (s[i - 1] + s[i + 1] + s[i - W] + s[i + W]) +
           wd * (s[i - W - 1] + s[i - W + 1] + s[i + W - 1] + s[i + W + 1]);
}

__device__ __forceinline__ bool interior(int X, int Y, int m) { return X >= 1 && X <= m - 1 && Y >= 1 && Y <= m - 1; }

// Thread -> node mapping of a W x W region in LDS for NT threads: each thread
// owns K vertically consecutive nodes of one column (segment), K chosen so
// that the segments cover the region with at most NT threads.  A 9-point
// stencil over a segment keeps a sliding 3 x 3 window in registers: (K+2)*3
// LDS reads for K nodes instead of 9K.
template <int W, int NT>
struct Seg {
    static constexpr int SPC = NT / W < 1 ? 1 : NT / W;    // segments per column
    static constexpr int K = (W + SPC - 1) / SPC;          // nodes per segment
    static constexpr int NS = W * ((W + K - 1) / K);       // segments in use
    int X, Y0;
    bool on;
    __device__ __forceinline__ Seg() {
        const int t = threadIdx.x;
        X = t % W;
        Y0 = (t / W) * K;
        on = t < NS;
    }
    __device__ __forceinline__ bool has(int k) const { return on && Y0 + k < W; }
    __device__ __forceinline__ int q(int k) const { return (Y0 + k) * W + X; }
};

// out[k] = (A x)(X, Y0 + k), same summation order as st9; rows and columns
// outside the region are clamped (their results are not used).
template <typename T, int W, int K>
__device__ __forceinline__ void st9_seg(const T* s, int X, int Y0, T wc, T we, T wd, T (&out)[K]) {
    const int xl = X > 0 ? X - 1 : 0, xr = X < W - 1 ? X + 1 : W - 1;
    auto row = [&](int y, T& l, T& c, T& r) {
        const int yy = y < 0 ? 0 : (y > W - 1 ? W - 1 : y);
        l = s[yy * W + xl];
        c = s[yy * W + X];
        r = s[yy * W + xr];
    };
    T l0, c0, r0, l1, c1, r1;
    row(Y0 - 1, l0, c0, r0);
    row(Y0, l1, c1, r1);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        T l2, c2, r2;
        row(Y0 + k + 1, l2, c2, r2);
        out[k] = wc * c1 + we * (l1 + r1 + c0 + c2) + wd * (l0 + r0 + l2 + r2);
        l0 = l1; c0 = c1; r0 = r1;
        l1 = l2; c1 = c2; r1 = r2;
    }
}

// Pre-smoothing from a zero guess on a W x W region: x_1 = c_r D^{-1} b, then
// NPRE-1 Chebyshev steps, step s updating [s, W-s).  The iterate is in LDS
// (sx, read by the stencil); b, the step direction and the iterate of the
// thread's nodes are in registers.
template <typename T, int W, int PPT, int NPRE>
__device__ __forceinline__ void pre_smooth(const T (&breg)[PPT], T (&d)[PPT], T (&xr)[PPT], T* sx, int FX0, int FY0,
                                           int m, const LevelDev& L, T wc, T we, T wd, T dinv) {
    const T cr0 = T(L.pre[0][1]);
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const int q = threadIdx.x + 256 * p;
        xr[p] = cr0 * dinv * breg[p];          // b is zero off the interior
        d[p] = xr[p];
        if (q < W * W) sx[q] = xr[p];
    }
    __syncthreads();
#pragma unroll
    for (int s = 1; s < NPRE; ++s) {
        const T cd = T(L.pre[s][0]), cr = T(L.pre[s][1]);
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            const int q = threadIdx.x + 256 * p;
            const int i = q % W, j = q / W;
            const int X = FX0 + i, Y = FY0 + j;
            if (q < W * W && i >= s && i < W - s && j >= s && j < W - s && X >= 1 && X <= m - 1 && Y >= 1 &&
                Y <= m - 1) {
                const T r = breg[p] - st9(sx, W, q, wc, we, wd);
                d[p] = cd * d[p] + cr * dinv * r;
                xr[p] += d[p];
            }
        }
        __syncthreads();
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            const int q = threadIdx.x + 256 * p;
            if (q < W * W) sx[q] = xr[p];
        }
        __syncthreads();
    }
}

template <typename T, int W, int PPT>
__device__ __forceinline__ void load_region(T (&breg)[PPT], const T* __restrict__ bcol, int FX0, int FY0, int m) {
    const int N1 = m + 1;
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const int q = threadIdx.x + 256 * p;
        const int X = FX0 + q % W, Y = FY0 + q / W;
        const bool inter = q < W * W && X >= 1 && X <= m - 1 && Y >= 1 && Y <= m - 1;
        breg[p] = inter ? bcol[Y * N1 + X] : T(0);
    }
}

// down: coarse tile of TC x TC coarse nodes starting at (I0, J0) = 1 + TC (tx, ty).
// Fine region: origin (2 I0 - 1 - NU, 2 J0 - 1 - NU), width W = 2 TC + 1 + 2 NU:
// pre-smoothing from zero (NU steps), residual, restriction b_c = P^T r.  The
// pre-smoothed iterate of the fine tile [2 I0 - 1, 2 I0 - 1 + 2 TC)^2 (interior
// nodes; the tiles cover the interior) is stored to xp ([column][(m+1)^2]) for
// the up kernel.
template <typename T, int TC, int NU>
__global__ __launch_bounds__(256) void k_mg_down(int m, const LevelDev* __restrict__ lev, int lvl,
                                                 const T* __restrict__ b, ColMap bmap, T* __restrict__ bc,
                                                 T* __restrict__ xp, int cpm, int tiles_x, Skip sk) {
    constexpr int W = 2 * TC + 1 + 2 * NU;
    constexpr int PPT = (W * W + 255) / 256;
    __shared__ T sx[W * W];
    const int c = blockIdx.y;
    if (sk.act && !sk.act[c / sk.cpv]) return;       // uniform per block, before any barrier
    const int tx = blockIdx.x % tiles_x, ty = blockIdx.x / tiles_x;
    const int I0 = 1 + tx * TC, J0 = 1 + ty * TC;
    const int ex = tx == 0 ? 1 : 0, ey = ty == 0 ? 1 : 0;     // also write the ring at index 0
    const int FX0 = 2 * I0 - 1 - NU, FY0 = 2 * J0 - 1 - NU;
    const int mc = m / 2;
    const LevelDev& L = lev[(c / cpm) * kMaxLevels + lvl];
    const T wc = T(L.wc), we = T(L.we), wd = T(L.wd), dinv = T(L.dinv);
    T breg[PPT], d[PPT], xr[PPT];
    load_region<T, W, PPT>(breg, b + bmap.off(c), FX0, FY0, m);
    pre_smooth<T, W, PPT, NU>(breg, d, xr, sx, FX0, FY0, m, L, wc, we, wd, dinv);
    {
        T* xpc = xp + (int64_t)c * (m + 1) * (m + 1);
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            const int q = threadIdx.x + 256 * p;
            const int i = q % W, j = q / W;
            const int X = FX0 + i, Y = FY0 + j;
            if (q < W * W && i >= NU && i < NU + 2 * TC && j >= NU && j < NU + 2 * TC && interior(X, Y, m))
                xpc[Y * (m + 1) + X] = xr[p];
        }
    }
    // residual on [NU, W-NU) (into registers, then over the iterate in LDS)
    T rr[PPT];
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const int q = threadIdx.x + 256 * p;
        const int i = q % W, j = q / W;
        const int X = FX0 + i, Y = FY0 + j;
        rr[p] = T(0);
        if (q < W * W && i >= NU && i < W - NU && j >= NU && j < W - NU && X >= 1 && X <= m - 1 && Y >= 1 &&
            Y <= m - 1)
            rr[p] = breg[p] - st9(sx, W, q, wc, we, wd);
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const int q = threadIdx.x + 256 * p;
        if (q < W * W) sx[q] = rr[p];
    }
    __syncthreads();
    // restriction (R = P^T: 1 centre, 1/2 edge partners, 1/4 corner partners)
    T* bco = bc + (int64_t)c * (mc + 1) * (mc + 1);
    for (int q = threadIdx.x; q < (TC + ex) * (TC + ey); q += blockDim.x) {
        const int I = I0 - ex + q % (TC + ex), J = J0 - ey + q / (TC + ex);
        if (I > mc || J > mc) continue;
        T v = T(0);
        if (I >= 1 && I <= mc - 1 && J >= 1 && J <= mc - 1) {
            const int i = 2 * I - FX0, j = 2 * J - FY0;
            const int pp = j * W + i;
            v = sx[pp] + T(0.5) * (sx[pp - 1] + sx[pp + 1] + sx[pp - W] + sx[pp + W]) +
                T(0.25) * (sx[pp - W - 1] + sx[pp - W + 1] + sx[pp + W - 1] + sx[pp + W + 1]);
        }
        bco[J * (mc + 1) + I] = v;
    }
}

// up: fine tile of TF x TF nodes starting at (X0, Y0) = 1 + TF (tx, ty), region
// with halo H = NPOST: the pre-smoothed iterate stored by the down kernel is
// read (zero off the interior), the interpolated coarse correction added, and
// NPOST post-smoothing steps run; the owned tile is written.
template <typename T, int TF, int NPOST>
__global__ __launch_bounds__(256) void k_mg_up(int m, const LevelDev* __restrict__ lev, int lvl,
                                               const T* __restrict__ ec, const T* __restrict__ b, ColMap bmap,
                                               const T* __restrict__ xp, T* __restrict__ xo, ColMap xomap, int cpm,
                                               int tiles_x, Skip sk) {
    constexpr int H0 = 0;
    constexpr int H = NPOST;
    constexpr int W = TF + 2 * H;
    constexpr int PPT = (W * W + 255) / 256;
    __shared__ T sx[W * W];
    const int c = blockIdx.y;
    if (sk.act && !sk.act[c / sk.cpv]) return;       // uniform per block, before any barrier
    const int tx = blockIdx.x % tiles_x, ty = blockIdx.x / tiles_x;
    const int FX0 = 1 + tx * TF - H, FY0 = 1 + ty * TF - H;
    const int ex = tx == 0 ? 1 : 0, ey = ty == 0 ? 1 : 0;
    const int mc = m / 2;
    const LevelDev& L = lev[(c / cpm) * kMaxLevels + lvl];
    const T wc = T(L.wc), we = T(L.we), wd = T(L.wd), dinv = T(L.dinv);
    const int N1 = m + 1, C1 = mc + 1;
    const T* ecol = ec + (int64_t)c * C1 * C1;
    // the coarse correction under the region, staged once in LDS (the
    // interpolation reads each coarse value up to nine times)
    constexpr int CW = W / 2 + 2;
    __shared__ T se[CW * CW];
    const int CX0 = FX0 >= 0 ? FX0 / 2 : -((1 - FX0) / 2), CY0 = FY0 >= 0 ? FY0 / 2 : -((1 - FY0) / 2);
    {
        constexpr int NE = (CW * CW + 255) / 256;
        T te[NE];
#pragma unroll
        for (int i = 0; i < NE; ++i) {      // loads first (clamped), masked stores after
            const int q = min((int)threadIdx.x + 256 * i, CW * CW - 1);
            te[i] = ecol[min(max(CY0 + q / CW, 0), mc) * C1 + min(max(CX0 + q % CW, 0), mc)];
        }
#pragma unroll
        for (int i = 0; i < NE; ++i) {
            const int q = threadIdx.x + 256 * i;
            const int I = CX0 + q % CW, J = CY0 + q / CW;
            if (q < CW * CW) se[q] = (I >= 0 && I <= mc && J >= 0 && J <= mc) ? te[i] : T(0);
        }
    }
    T breg[PPT], d[PPT], xr[PPT];
    load_region<T, W, PPT>(breg, b + bmap.off(c), FX0, FY0, m);
    load_region<T, W, PPT>(xr, xp + (int64_t)c * N1 * N1, FX0, FY0, m);
    __syncthreads();                    // se complete
    // x += P e_c on the region's interior nodes
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const int q = threadIdx.x + 256 * p;
        const int i = q % W, j = q / W;
        const int X = FX0 + i, Y = FY0 + j;
        if (q < W * W && i >= H0 && i < W - H0 && j >= H0 && j < W - H0 && X >= 1 && X <= m - 1 && Y >= 1 &&
            Y <= m - 1) {
            const int I0 = (X >> 1) - CX0, J0 = (Y >> 1) - CY0, I1 = I0 + (X & 1), J1 = J0 + (Y & 1);
            xr[p] += T(0.25) * (se[J0 * CW + I0] + se[J0 * CW + I1] + se[J1 * CW + I0] + se[J1 * CW + I1]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const int q = threadIdx.x + 256 * p;
        if (q < W * W) sx[q] = xr[p];
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < NPOST; ++s) {
        const T cd = T(L.post[s][0]), cr = T(L.post[s][1]);
        const int lo = H0 + s + 1, hi = W - H0 - s - 1;
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            const int q = threadIdx.x + 256 * p;
            const int i = q % W, j = q / W;
            const int X = FX0 + i, Y = FY0 + j;
            if (q < W * W && i >= lo && i < hi && j >= lo && j < hi && X >= 1 && X <= m - 1 && Y >= 1 &&
                Y <= m - 1) {
                const T r = breg[p] - st9(sx, W, q, wc, we, wd);
                d[p] = (s == 0 ? T(0) : cd * d[p]) + cr * dinv * r;
                xr[p] += d[p];
            }
        }
        if (s + 1 < NPOST) {
            __syncthreads();
#pragma unroll
            for (int p = 0; p < PPT; ++p) {
                const int q = threadIdx.x + 256 * p;
                if (q < W * W) sx[q] = xr[p];
            }
            __syncthreads();
        }
    }
    T* out = xo + xomap.off(c);
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const int q = threadIdx.x + 256 * p;
        const int X = FX0 + q % W, Y = FY0 + q / W;
        if (q < W * W && X >= FX0 + H - ex && X < FX0 + H + TF && Y >= FY0 + H - ey && Y < FY0 + H + TF &&
            X <= m && Y <= m)
            out[Y * N1 + X] = xr[p];
    }
}

// Chebyshev semi-iteration on the mass matrix for the state and control
// blocks, all steps in LDS (halo = steps - 1 nodes).  Column l of vector v
// (l < 2 nt n_xi) is r[v*vstride + l*nodes ...]; the last step writes
// z = x / (s tau D_t) with s = 1 (mean column) or 1+gamma (state), beta (control).
struct ChebW {
    float pad;
    double omega[16];   // omega_{k+1} for k = 1..steps-1
};

template <typename T, int TF, int H, int NT>
__global__ __launch_bounds__(NT) void k_mass_cheb_fused(int n, int nxi, int nt, int time, int64_t nodes, OpDev op,
                                                         int64_t vstride, const T* __restrict__ r, T* __restrict__ z,
                                                         ChebW cw, int tiles_x, int64_t zstride, int l0, int cpg,
                                                         int gstride) {
    // H = steps - 1 stencil steps; the region keeps a halo of at least one node
    // so that the first tile row and column also hold the ring at index 0
    constexpr int HR = H > 0 ? H : 1;
    constexpr int W = TF + 2 * HR;
    using SG = Seg<W, NT>;
    constexpr int K = SG::K;
    __shared__ T sA[W * W];           // x_k (read by the mass stencil), two copies: one barrier per step
    __shared__ T sB[W * W];
    const SG g;
    // column of [y | u] (n_t n_xi state columns, then control): groups of cpg
    // consecutive columns, gstride columns apart
    const int l = l0 + (int)(blockIdx.y / cpg) * gstride + (int)(blockIdx.y % cpg);
    const int vec = blockIdx.z;
    if (op.active && !op.active[vec]) return;        // uniform per block, before any barrier
    const int mem = op.mem_shared ? 0 : vec;
    const int tx = blockIdx.x % tiles_x, ty = blockIdx.x / tiles_x;
    const int FX0 = 1 + tx * TF - HR, FY0 = 1 + ty * TF - HR;
    const int ex = tx == 0 ? 1 : 0, ey = ty == 0 ? 1 : 0;
    const int N1 = n + 1;
    const T h = T(1) / T(n);
    const T h2_36 = h * h / T(36);
    const T dinv = T(1) / (T(1.25) * T(4) * h * h / T(9));
    const T* rc = r + (int64_t)vec * vstride + (int64_t)l * nodes;
    T breg[K], xp[K], xc[K];          // b, x_{k-1}, x_k of the thread's nodes
    // all loads first (clamped addresses, masked after), so that they are in
    // flight together rather than one per LDS write
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int X = FX0 + g.X, Y = FY0 + g.Y0 + k;
        breg[k] = rc[min(max(Y, 0), n) * N1 + min(max(X, 0), n)];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int X = FX0 + g.X, Y = FY0 + g.Y0 + k;
        breg[k] = g.has(k) && interior(X, Y, n) ? breg[k] : T(0);
        xp[k] = T(0);                 // x_0
        xc[k] = dinv * breg[k];       // x_1 (omega_1 = 1)
        if (g.has(k)) sA[g.q(k)] = xc[k];
    }
    __syncthreads();
    T* cur = sA;
    T* nxt = sB;
#pragma unroll 1
    for (int s = 1; s <= H; ++s) {
        const T om = T(cw.omega[s - 1]);
        const int lo = s, hi = W - s;
        T mx[K];
        // mass stencil (h^2/36) [1 4 1; 4 16 4; 1 4 1]
        st9_seg<T, W, K>(cur, g.X, g.Y0, T(16), T(4), T(1), mx);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int i = g.X, j = g.Y0 + k;
            if (g.has(k) && i >= lo && i < hi && j >= lo && j < hi && interior(FX0 + i, FY0 + j, n)) {
                const T Mx = h2_36 * mx[k];
                const T v = om * (dinv * (breg[k] - Mx) + xc[k] - xp[k]) + xp[k];
                xp[k] = xc[k];
                xc[k] = v;
            }
            if (s < H && g.has(k)) nxt[g.q(k)] = xc[k];
        }
        if (s < H) {
            __syncthreads();
            T* tmp = cur;
            cur = nxt;
            nxt = tmp;
        }
    }
    const MemberDev md = op.mem[mem];
    const int var = l / (nt * nxi);
    const int t = (l / nxi) % nt;
    const int j = l % nxi;
    const T Dt = (time && (t == 0 || t == nt - 1)) ? T(0.5) : T(1);
    const T sc_ = var == 0 ? (j == 0 ? T(1) : T(md.hg)) : T(md.beta);
    const T f = T(1) / (sc_ * T(md.tau) * Dt);
    T* zc = z + (int64_t)vec * zstride + (int64_t)l * nodes;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int X = FX0 + g.X, Y = FY0 + g.Y0 + k;
        if (g.has(k) && X >= FX0 + HR - ex && X < FX0 + HR + TF && Y >= FY0 + HR - ey && Y < FY0 + HR + TF &&
            X <= n && Y <= n)
            zc[Y * N1 + X] = f * xc[k];
    }
}

// --------------------------------------------------------------------------
// Coarse end of the V-cycle in one workgroup per column.  Levels M0, M0/2, ..,
// kCoarseN live in LDS (right-hand side and iterate per level, one residual
// buffer): pre-smoothing from zero, residual and restriction on the way down,
// the direct solve on the kCoarseN grid (dense inverse of the interior
// operator), interpolation and post-smoothing on the way up.  Replaces
// 2 log2(M0/kCoarseN) + 1 launches per V-cycle by one.  Each level is a
// template instance (compile-time width); a thread's nodes are a vertical
// segment (Seg) whose b, iterate and step direction stay in registers.
// --------------------------------------------------------------------------
constexpr int kTailThreads = 1024;   // 512 or 256 measured slower (bit-identical)

__host__ __device__ constexpr int tail_levels(int m0) { return m0 <= kCoarseN ? 1 : 1 + tail_levels(m0 / 2); }
__host__ __device__ constexpr int tail_offset(int m0, int k) {
    return k == 0 ? 0 : (m0 + 1) * (m0 + 1) + tail_offset(m0 / 2, k - 1);
}
// offset of level m in the per-level arrays of a tail starting at m0
__host__ __device__ constexpr int level_offset(int m0, int m) { return m0 == m ? 0 : (m0 + 1) * (m0 + 1) + level_offset(m0 / 2, m); }
__host__ __device__ constexpr int level_index(int m0, int m) { return m0 == m ? 0 : 1 + level_index(m0 / 2, m); }

template <typename T, int M0>
struct TailLds {
    static constexpr int NL = tail_levels(M0);
    static constexpr int W0 = M0 + 1;
    static constexpr int total = tail_offset(M0, NL);    // sum of (m+1)^2 over the levels
    T b[total];
    T x[total];
    T r[W0 * W0];
};

// One Chebyshev step from buffer `in` to buffer `out` (ping-pong: a single
// barrier per step): d = c_d d + c_r D^{-1} (b - A x), x += d on interior nodes.
template <typename T, int W, int K>
__device__ __forceinline__ void tail_step(const Seg<W, kTailThreads>& g, const T* in, T* out, int m, const T (&breg)[K],
                                          T (&d)[K], T (&xr)[K], T wc, T we, T wd, T dinv, T cd, T cr, bool first) {
    T ax[K];
    st9_seg<T, W, K>(in, g.X, g.Y0, wc, we, wd, ax);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (g.has(k) && interior(g.X, g.Y0 + k, m)) {
            d[k] = (first ? T(0) : cd * d[k]) + cr * dinv * (breg[k] - ax[k]);
            xr[k] += d[k];
        }
        if (g.has(k)) out[g.q(k)] = xr[k];
    }
    __syncthreads();
}

// down at level M: pre-smoothing from zero, residual, restriction to level M/2.
// The iterate ping-pongs between the level's array P and the shared buffer
// Q = s.r so that the final pre-smoothed iterate lands in P (kept for the up
// sweep); the first stencil step is taken straight from b (x_1 = c_r D^{-1} b).
template <typename T, int M, int M0>
__device__ __forceinline__ void tail_down(TailLds<T, M0>& s, const LevelDev* slev, int npre) {
    constexpr int W = M + 1, mc = M / 2, C1 = mc + 1;
    using SG = Seg<W, kTailThreads>;
    constexpr int K = SG::K;
    const SG g;
    const T* B = s.b + level_offset(M0, M);
    T* P = s.x + level_offset(M0, M);
    T* Q = s.r;
    T* Bc = s.b + level_offset(M0, mc);
    const LevelDev& L = slev[level_index(M0, M)];
    const T wc = T(L.wc), we = T(L.we), wd = T(L.wd), dinv = T(L.dinv);
    const T c1 = T(L.pre[0][1]) * dinv;
    T breg[K], d[K], xr[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        breg[k] = g.has(k) ? B[g.q(k)] : T(0);   // zero off the interior
        xr[k] = c1 * breg[k];
        d[k] = xr[k];
    }
    if (npre == 1) {
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (g.has(k)) P[g.q(k)] = xr[k];
        __syncthreads();
    } else {
        // step 1 from b: A x_1 = c_1 A b; then steps 2..npre-1 alternate so that
        // step npre-1 writes P
        {
            const T cd = T(L.pre[1][0]), cr = T(L.pre[1][1]);
            T ab[K];
            st9_seg<T, W, K>(B, g.X, g.Y0, wc, we, wd, ab);
            T* out = (npre - 1) % 2 == 1 ? P : Q;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (g.has(k) && interior(g.X, g.Y0 + k, M)) {
                    d[k] = cd * d[k] + cr * dinv * (breg[k] - c1 * ab[k]);
                    xr[k] += d[k];
                }
                if (g.has(k)) out[g.q(k)] = xr[k];
            }
            __syncthreads();
        }
        for (int st = 2; st < npre; ++st) {
            const bool to_p = (npre - 1 - st) % 2 == 0;
            tail_step<T, W, K>(g, to_p ? Q : P, to_p ? P : Q, M, breg, d, xr, wc, we, wd, dinv, T(L.pre[st][0]),
                               T(L.pre[st][1]), false);
        }
    }
    {
        T ax[K];
        st9_seg<T, W, K>(P, g.X, g.Y0, wc, we, wd, ax);
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (g.has(k)) Q[g.q(k)] = interior(g.X, g.Y0 + k, M) ? breg[k] - ax[k] : T(0);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < C1 * C1; q += kTailThreads) {
        const int I = q % C1, J = q / C1;
        T v = T(0);
        if (I >= 1 && I <= mc - 1 && J >= 1 && J <= mc - 1) {
            const int pf = 2 * J * W + 2 * I;
            v = Q[pf] + T(0.5) * (Q[pf - 1] + Q[pf + 1] + Q[pf - W] + Q[pf + W]) +
                T(0.25) * (Q[pf - W - 1] + Q[pf - W + 1] + Q[pf + W - 1] + Q[pf + W + 1]);
        }
        Bc[q] = v;
    }
    __syncthreads();
    if constexpr (mc > kCoarseN) tail_down<T, mc, M0>(s, slev, npre);
}

// up at level M (coarser levels first): x += P e (pointwise, in place or into
// Q), then post-smoothing steps alternating so that the last one writes P.
template <typename T, int M, int M0>
__device__ __forceinline__ void tail_up(TailLds<T, M0>& s, const LevelDev* slev, int npost) {
    constexpr int W = M + 1, mc = M / 2, C1 = mc + 1;
    if constexpr (mc > kCoarseN) tail_up<T, mc, M0>(s, slev, npost);
    using SG = Seg<W, kTailThreads>;
    constexpr int K = SG::K;
    const SG g;
    const T* B = s.b + level_offset(M0, M);
    T* P = s.x + level_offset(M0, M);
    T* Q = s.r;
    const T* E = s.x + level_offset(M0, mc);
    const LevelDev& L = slev[level_index(M0, M)];
    const T wc = T(L.wc), we = T(L.we), wd = T(L.wd), dinv = T(L.dinv);
    T breg[K], d[K], xr[K];
    T* first = npost % 2 == 0 ? P : Q;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        breg[k] = d[k] = xr[k] = T(0);
        if (g.has(k)) {
            const int X = g.X, Y = g.Y0 + k;
            breg[k] = B[g.q(k)];
            xr[k] = P[g.q(k)];
            if (interior(X, Y, M)) {
                const int I0 = X >> 1, J0 = Y >> 1, I1 = I0 + (X & 1), J1 = J0 + (Y & 1);
                xr[k] += T(0.25) * (E[J0 * C1 + I0] + E[J0 * C1 + I1] + E[J1 * C1 + I0] + E[J1 * C1 + I1]);
            }
            first[g.q(k)] = xr[k];
        }
    }
    __syncthreads();
    for (int st = 0; st < npost; ++st) {
        const bool to_p = (npost - 1 - st) % 2 == 0;
        tail_step<T, W, K>(g, to_p ? Q : P, to_p ? P : Q, M, breg, d, xr, wc, we, wd, dinv, T(L.post[st][0]),
                           T(L.post[st][1]), st == 0);
    }
}

template <typename T, int M0>
__global__ __launch_bounds__(kTailThreads) void k_mg_tail(const LevelDev* __restrict__ lev, int lvl0, int npre,
                                                          int npost, const T* __restrict__ b, ColMap bmap,
                                                          T* __restrict__ x, ColMap xmap, const T* __restrict__ ainv,
                                                          int cpm, Skip sk) {
    using Lds = TailLds<T, M0>;
    constexpr int NL = Lds::NL;
    constexpr int W0 = Lds::W0;
    constexpr int CN1 = kCoarseN + 1, CNU = (kCoarseN - 1) * (kCoarseN - 1);
    __shared__ Lds s;
    __shared__ LevelDev slev[NL > 1 ? NL - 1 : 1];
    __shared__ T sA[CNU * CNU];             // interior block of the coarse inverse
    const int c = blockIdx.x;
    if (sk.act && !sk.act[c / sk.cpv]) return;       // uniform per block, before any barrier
    const int mem = c / cpm;
    // issue every global read first, into registers (clamped addresses): the
    // column, the level parameters and the coarse inverse (consumed only after
    // the down sweep); then mask and store them to LDS
    const T* bcol = b + bmap.off(c);
    constexpr int NB = (W0 * W0 + kTailThreads - 1) / kTailThreads;
    constexpr int NA = (CNU * CNU + kTailThreads - 1) / kTailThreads;
    constexpr int LW = sizeof(LevelDev) / sizeof(double);
    const T* A = ainv + (int64_t)mem * kCoarsePad * kCoarsePad;
    T rb[NB], ra[NA];
#pragma unroll
    for (int i = 0; i < NB; ++i) rb[i] = bcol[min((int)threadIdx.x + i * kTailThreads, W0 * W0 - 1)];
#pragma unroll
    for (int i = 0; i < NA; ++i) {
        const int q = min((int)threadIdx.x + i * kTailThreads, CNU * CNU - 1);
        ra[i] = A[(q / CNU) * kCoarsePad + q % CNU];
    }
    for (int q = threadIdx.x; q < (NL - 1) * LW; q += kTailThreads)
        ((double*)slev)[q] = ((const double*)(lev + mem * kMaxLevels + lvl0))[q];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int q = threadIdx.x + i * kTailThreads;
        if (q < W0 * W0) s.b[q] = interior(q % W0, q / W0, M0) ? rb[i] : T(0);
    }
#pragma unroll
    for (int i = 0; i < NA; ++i) {
        const int q = threadIdx.x + i * kTailThreads;
        if (q < CNU * CNU) sA[q] = ra[i];
    }
    __syncthreads();
    tail_down<T, M0, M0>(s, slev, npre);
    // direct solve on the kCoarseN grid: four threads per interior unknown
    {
        const int row = threadIdx.x / 4, part = threadIdx.x % 4;
        const T* Bc = s.b + tail_offset(M0, NL - 1);
        T* Xc = s.x + tail_offset(M0, NL - 1);
        T acc = T(0);
        if (row < CNU) {
            for (int k = part; k < CNU; k += 4) {
                const int ix = k % (kCoarseN - 1) + 1, iy = k / (kCoarseN - 1) + 1;
                acc += sA[row * CNU + k] * Bc[iy * CN1 + ix];
            }
        }
        acc += __shfl_xor(acc, 1, 64);
        acc += __shfl_xor(acc, 2, 64);
        for (int q = threadIdx.x; q < CN1 * CN1; q += kTailThreads) Xc[q] = T(0);
        __syncthreads();
        if (row < CNU && part == 0) {
            const int ix = row % (kCoarseN - 1) + 1, iy = row / (kCoarseN - 1) + 1;
            Xc[iy * CN1 + ix] = acc;
        }
        __syncthreads();
    }
    tail_up<T, M0, M0>(s, slev, npost);
    T* xcol = x + xmap.off(c);
    for (int q = threadIdx.x; q < W0 * W0; q += kTailThreads) xcol[q] = s.x[q];
}

template <typename T, int M0>
void tail_m(const LevelDev* lev, int lvl0, int npre, int npost, const T* b, ColMap bmap, T* x, ColMap xmap,
            const T* ainv, int ncols, int cpm, Skip sk, hipStream_t st) {
    hipLaunchKernelGGL((k_mg_tail<T, M0>), dim3(ncols), dim3(kTailThreads), 0, st, lev, lvl0, npre, npost, b, bmap,
                       x, xmap, ainv, cpm, sk);
}

template <typename T, int H>
void cheb_h(const Shape& s, const OpDev& op, const T* r, int64_t rstride, T* z, int64_t zstride, int l0, int ncols,
            int ngrp, int gstride, int nvec, const ChebW& cw, hipStream_t st) {
    if ((int64_t)ncols * ngrp > 65535 || nvec > 65535) throw Error(SG_ERR_INVALID, "Chebyshev: launch grid too large");
    // 32-node tiles at every grid size: 64-node tiles (512 threads) fetch fewer
    // halo nodes but measured slower at 128^2 and 512^2
    constexpr int TF = 32;
    const int tx = (s.n - 1 + TF - 1) / TF;
    hipLaunchKernelGGL((k_mass_cheb_fused<T, TF, H, 256>), dim3(tx * tx, ncols * ngrp, nvec), dim3(256), 0, st, s.n,
                       s.nxi, s.nt, (int)s.time, s.nodes, op, rstride, r, z, cw, tx, zstride, l0, ncols, gstride);
}

constexpr int TCD = 16;   // coarse nodes per down tile side
constexpr int TFU = 32;   // fine nodes per up tile side
// Launches with fewer workgroups than this at the tile sizes above (a few
// columns on a level) take half-size tiles instead: the launch then lasts
// about one workgroup's chain of barriered steps, which halves with the tile.
// Every node's arithmetic is the same in either tiling.
constexpr int64_t kSmallTileBlocks = 512;

template <typename T, int NU>
void down_nu(int m, const LevelDev* lev, int lvl, const T* b, ColMap bmap, T* bc, T* xp, int ncols, int cpm, Skip sk,
             hipStream_t st) {
    const int mc = m / 2;
    const int tx = (mc - 1 + TCD - 1) / TCD;
    if ((int64_t)tx * tx * ncols < kSmallTileBlocks) {
        constexpr int TC = TCD / 2;
        const int ts = (mc - 1 + TC - 1) / TC;
        hipLaunchKernelGGL((k_mg_down<T, TC, NU>), dim3(ts * ts, ncols), dim3(256), 0, st, m, lev, lvl, b, bmap, bc,
                           xp, cpm, ts, sk);
        return;
    }
    hipLaunchKernelGGL((k_mg_down<T, TCD, NU>), dim3(tx * tx, ncols), dim3(256), 0, st, m, lev, lvl, b, bmap, bc, xp,
                       cpm, tx, sk);
}

template <typename T, int NPOST>
void up_nu(int m, const LevelDev* lev, int lvl, const T* ec, const T* b, ColMap bmap, const T* xp, T* xo,
           ColMap xomap, int ncols, int cpm, Skip sk, hipStream_t st) {
    const int tx = (m - 1 + TFU - 1) / TFU;
    if ((int64_t)tx * tx * ncols < kSmallTileBlocks) {
        constexpr int TF = TFU / 2;
        const int ts = (m - 1 + TF - 1) / TF;
        hipLaunchKernelGGL((k_mg_up<T, TF, NPOST>), dim3(ts * ts, ncols), dim3(256), 0, st, m, lev, lvl, ec, b, bmap,
                           xp, xo, xomap, cpm, ts, sk);
        return;
    }
    hipLaunchKernelGGL((k_mg_up<T, TFU, NPOST>), dim3(tx * tx, ncols), dim3(256), 0, st, m, lev, lvl, ec, b, bmap, xp,
                       xo, xomap, cpm, tx, sk);
}

}  // namespace

template <typename T>
void launch_mg_down(int m, const LevelDev* lev, int lvl, int npre, const T* b, ColMap bmap, T* bc, T* xp, int ncols,
                    int cpm, const int* act, int cpv, hipStream_t st) {
    if (ncols > 65535) throw Error(SG_ERR_INVALID, "multigrid: too many columns in one launch");
    const Skip sk{act, cpv};
    switch (npre) {
        case 1: down_nu<T, 1>(m, lev, lvl, b, bmap, bc, xp, ncols, cpm, sk, st); break;
        case 2: down_nu<T, 2>(m, lev, lvl, b, bmap, bc, xp, ncols, cpm, sk, st); break;
        case 3: down_nu<T, 3>(m, lev, lvl, b, bmap, bc, xp, ncols, cpm, sk, st); break;
        case 4: down_nu<T, 4>(m, lev, lvl, b, bmap, bc, xp, ncols, cpm, sk, st); break;
        default: throw Error(SG_ERR_INVALID, "smoothing degree must be 1..4");
    }
    SG_HIP(hipGetLastError());
}

template <typename T>
void launch_mg_up(int m, const LevelDev* lev, int lvl, int npost, const T* ec, const T* b, ColMap bmap, const T* xp,
                  T* xo, ColMap xomap, int ncols, int cpm, const int* act, int cpv, hipStream_t st) {
    if (ncols > 65535) throw Error(SG_ERR_INVALID, "multigrid: too many columns in one launch");
    const Skip sk{act, cpv};
    switch (npost) {
        case 1: up_nu<T, 1>(m, lev, lvl, ec, b, bmap, xp, xo, xomap, ncols, cpm, sk, st); break;
        case 2: up_nu<T, 2>(m, lev, lvl, ec, b, bmap, xp, xo, xomap, ncols, cpm, sk, st); break;
        case 3: up_nu<T, 3>(m, lev, lvl, ec, b, bmap, xp, xo, xomap, ncols, cpm, sk, st); break;
        case 4: up_nu<T, 4>(m, lev, lvl, ec, b, bmap, xp, xo, xomap, ncols, cpm, sk, st); break;
        default: throw Error(SG_ERR_INVALID, "smoothing degree must be 1..4");
    }
    SG_HIP(hipGetLastError());
}

template <typename T>
void launch_mg_tail(int m0, const LevelDev* lev, int lvl0, int npre, int npost, const T* b, ColMap bmap, T* x,
                    ColMap xmap, const T* ainv, int ncols, int cpm, const int* act, int cpv, hipStream_t st) {
    if (ncols < 1) return;
    const Skip sk{act, cpv};
    if (npre < 1 || npre > kMaxSmooth || npost < 0 || npost > kMaxSmooth)
        throw Error(SG_ERR_INVALID, "smoothing degree must be 1..4");
    switch (m0) {
        case 16: tail_m<T, 16>(lev, lvl0, npre, npost, b, bmap, x, xmap, ainv, ncols, cpm, sk, st); break;
        case 32: tail_m<T, 32>(lev, lvl0, npre, npost, b, bmap, x, xmap, ainv, ncols, cpm, sk, st); break;
        case 64: tail_m<T, 64>(lev, lvl0, npre, npost, b, bmap, x, xmap, ainv, ncols, cpm, sk, st); break;
        default: throw Error(SG_ERR_INVALID, "multigrid tail level must be 16, 32 or 64");
    }
    SG_HIP(hipGetLastError());
}

// Returns false when the step count has no fused kernel (more than 9 steps).
template <typename T>
bool launch_mass_cheb_fused(const Shape& s, const OpDev& op, const T* r, T* z, int nvec, int steps, hipStream_t st) {
    return launch_mass_cheb_cols<T>(s, op, r, 3 * s.blk, z, 3 * s.blk, 0, 2 * s.nt * s.nxi, 1, 0, nvec, steps, st);
}

template <typename T>
bool launch_mass_cheb_cols(const Shape& s, const OpDev& op, const T* r, int64_t rstride, T* z, int64_t zstride, int l0,
                           int ncols, int ngrp, int gstride, int nvec, int steps, hipStream_t st) {
    if (steps < 1 || steps > 9) return false;
    ChebW cw{};
    const double rho = 0.8;
    double omega = 1.0;
    for (int k = 1; k < steps; ++k) {
        omega = (k == 1) ? 1.0 / (1.0 - 0.5 * rho * rho) : 1.0 / (1.0 - 0.25 * rho * rho * omega);
        cw.omega[k - 1] = omega;
    }
    switch (steps - 1) {
        case 0: cheb_h<T, 0>(s, op, r, rstride, z, zstride, l0, ncols, ngrp, gstride, nvec, cw, st); break;
        case 1: cheb_h<T, 1>(s, op, r, rstride, z, zstride, l0, ncols, ngrp, gstride, nvec, cw, st); break;
        case 2: cheb_h<T, 2>(s, op, r, rstride, z, zstride, l0, ncols, ngrp, gstride, nvec, cw, st); break;
        case 3: cheb_h<T, 3>(s, op, r, rstride, z, zstride, l0, ncols, ngrp, gstride, nvec, cw, st); break;
        case 4: cheb_h<T, 4>(s, op, r, rstride, z, zstride, l0, ncols, ngrp, gstride, nvec, cw, st); break;
        case 5: cheb_h<T, 5>(s, op, r, rstride, z, zstride, l0, ncols, ngrp, gstride, nvec, cw, st); break;
        case 6: cheb_h<T, 6>(s, op, r, rstride, z, zstride, l0, ncols, ngrp, gstride, nvec, cw, st); break;
        case 7: cheb_h<T, 7>(s, op, r, rstride, z, zstride, l0, ncols, ngrp, gstride, nvec, cw, st); break;
        default: cheb_h<T, 8>(s, op, r, rstride, z, zstride, l0, ncols, ngrp, gstride, nvec, cw, st); break;
    }
    SG_HIP(hipGetLastError());
    return true;
}

template bool launch_mass_cheb_fused<double>(const Shape&, const OpDev&, const double*, double*, int, int, hipStream_t);
template bool launch_mass_cheb_fused<float>(const Shape&, const OpDev&, const float*, float*, int, int, hipStream_t);
template bool launch_mass_cheb_cols<double>(const Shape&, const OpDev&, const double*, int64_t, double*, int64_t, int,
                                            int, int, int, int, int, hipStream_t);
template bool launch_mass_cheb_cols<float>(const Shape&, const OpDev&, const float*, int64_t, float*, int64_t, int, int,
                                           int, int, int, int, hipStream_t);

template void launch_mg_tail<double>(int, const LevelDev*, int, int, int, const double*, ColMap, double*, ColMap,
                                     const double*, int, int, const int*, int, hipStream_t);
template void launch_mg_tail<float>(int, const LevelDev*, int, int, int, const float*, ColMap, float*, ColMap,
                                    const float*, int, int, const int*, int, hipStream_t);
template void launch_mg_down<double>(int, const LevelDev*, int, int, const double*, ColMap, double*, double*, int,
                                     int, const int*, int, hipStream_t);
template void launch_mg_down<float>(int, const LevelDev*, int, int, const float*, ColMap, float*, float*, int, int,
                                    const int*, int, hipStream_t);
template void launch_mg_up<double>(int, const LevelDev*, int, int, const double*, const double*, ColMap,
                                   const double*, double*, ColMap, int, int, const int*, int, hipStream_t);
template void launch_mg_up<float>(int, const LevelDev*, int, int, const float*, const float*, ColMap, const float*,
                                  float*, ColMap, int, int, const int*, int, hipStream_t);

}  // namespace sg
