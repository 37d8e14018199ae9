// SG operator, KKT apply and hGS right-hand sides for a coefficient with a
// general chaos coupling (the log-normal field of Section 5): A = sum_l H_l
// (x) A_l with dense-pattern H_l, intra-level couplings included.
//
// On element e the operator's chaos coupling is B_e = sum_l kappa_l(e) H_l
// (nxi x nxi, precomputed per member), and A_l = sum_e kappa_l(e) K_e with one
// reference Q1 stiffness, so
//   (A X)_j(node) = sum_{e at node} sum_i B_e[i][j] (K_ref X_i|e)(node),
// where the corner value of the reference stiffness is (4 v_a - v_b - v_c -
// 2 v_opp) / 6 (b, c the edge neighbours, opp the diagonal corner).  One
// thread owns one node and a chunk of output columns: for every input column
// it loads the 3 x 3 node neighbourhood once, forms the four element corner
// values and accumulates them with the four elements' B entries of its output
// columns (B is read from cache: four neighbouring nodes share an element).
#include "common.hpp"

namespace sg {

namespace {

constexpr int GJC = 8;     // output columns per thread
constexpr int GTX = 16;    // node tile (GTX x GTX threads per block)

// out_j = base_j + s * sum_{i in [ilo1, ihi1) u [ilo2, ihi2)} sum_e (B_e[i][j] + [i == j] mean_c) kr_e(X_i)
// for the L output columns j = j0 .. j0+L-1 of each slice (vector, t); s =
// scale, or -scale_off * off_scale of the slice's member when scale_off != 0 (1:
// subtract the couplings, -1: add them); base may be null.
// X: field blocks with member stride xms and time stride xts ([t][i][node]).
template <typename T>
__global__ __launch_bounds__(GTX* GTX) void k_gen_sg(int n, int nxi, int nt, const double* __restrict__ B, int64_t bms,
                                                     const T* __restrict__ X, int64_t xms, int64_t xts, int ilo1,
                                                     int ihi1, int ilo2, int ihi2, int j0, int L,
                                                     const T* __restrict__ base, ColMap bmap, T* __restrict__ out,
                                                     ColMap omap, double scale, int scale_off, double mean_c,
                                                     const MemberDev* __restrict__ mem, int shared,
                                                     const int* __restrict__ act, int tiles_x) {
    const int slice = blockIdx.z;
    const int vec = slice / nt, t = slice % nt;
    if (act && !act[vec]) return;
    const int ix = (blockIdx.x % tiles_x) * GTX + threadIdx.x % GTX;
    const int iy = (blockIdx.x / tiles_x) * GTX + threadIdx.x / GTX;
    if (ix > n || iy > n) return;
    const int N1 = n + 1;
    const int64_t q = (int64_t)iy * N1 + ix;
    const int l0 = blockIdx.y * GJC;
    const int cnt = min(GJC, L - l0);
    const int64_t cbase = (int64_t)slice * L + l0;        // output column index of (slice, l0)
    if (ix == 0 || iy == 0 || ix == n || iy == n) {
        for (int c = 0; c < cnt; ++c) out[omap.off((int)(cbase + c)) + q] = T(0);
        return;
    }
    const int mm = shared ? 0 : vec;
    const double s = scale_off ? -(double)scale_off * mem[mm].off_scale : scale;
    const double* Bm = B + (int64_t)mm * bms;
    const int64_t nn = (int64_t)nxi * nxi;
    // the four elements at the node: (ex, ey) = (ix-1, iy-1), (ix, iy-1), (ix-1, iy), (ix, iy)
    const double* Be[4] = {Bm + ((int64_t)(iy - 1) * n + (ix - 1)) * nn, Bm + ((int64_t)(iy - 1) * n + ix) * nn,
                           Bm + ((int64_t)iy * n + (ix - 1)) * nn, Bm + ((int64_t)iy * n + ix) * nn};
    double acc[GJC];
#pragma unroll
    for (int c = 0; c < GJC; ++c) acc[c] = 0.0;
    const T* Xs = X + (int64_t)vec * xms + (int64_t)t * xts;
    for (int r = 0; r < 2; ++r) {
        const int ilo = r == 0 ? ilo1 : ilo2, ihi = r == 0 ? ihi1 : ihi2;
        for (int i = ilo; i < ihi; ++i) {
            const T* xi = Xs + (int64_t)i * N1 * N1;
            double v[3][3];          // the ring holds no unknowns: its values count as zero
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) {
                    const int jx = ix + dx - 1, jy = iy + dy - 1;
                    const bool in = jx > 0 && jx < n && jy > 0 && jy < n;
                    const T xv = xi[q + (int64_t)(dy - 1) * N1 + (dx - 1)];
                    v[dy][dx] = in ? (double)xv : 0.0;
                }
            const double a = 4.0 * v[1][1];
            // corner values of the reference stiffness in the four elements
            const double kr[4] = {(a - v[1][0] - v[0][1] - 2.0 * v[0][0]) / 6.0,
                                  (a - v[1][2] - v[0][1] - 2.0 * v[0][2]) / 6.0,
                                  (a - v[1][0] - v[2][1] - 2.0 * v[2][0]) / 6.0,
                                  (a - v[1][2] - v[2][1] - 2.0 * v[2][2]) / 6.0};
#pragma unroll
            for (int c = 0; c < GJC; ++c) {
                if (c < cnt) {
                    const int j = j0 + l0 + c;
                    const int64_t o = (int64_t)i * nxi + j;
                    double b = Be[0][o] * kr[0] + Be[1][o] * kr[1] + Be[2][o] * kr[2] + Be[3][o] * kr[3];
                    if (i == j) b += mean_c * (kr[0] + kr[1] + kr[2] + kr[3]);
                    acc[c] += b;
                }
            }
        }
    }
#pragma unroll
    for (int c = 0; c < GJC; ++c) {
        if (c < cnt) {
            const int col = (int)(cbase + c);
            const double bv = base ? (double)base[bmap.off(col) + q] : 0.0;
            out[omap.off(col) + q] = (T)(bv + s * acc[c]);
        }
    }
}

// KKT rows from the two stiffness products T1 = A Lambda, T2 = A Y (per
// (vector, t) slice, [t][j][node] blocks of member stride blk):
//   steady: R^Y = M_gamma Y - T1, R^U = beta M U + M Lambda, R^L = -T2 + M U;
//   time:   R^Y_t = tau D_t M_gamma Y_t - (M L_t + tau T1_t) + M L_{t+1},
//           R^U_t = beta tau D_t M U_t + tau M L_t,
//           R^L_t = -(M Y_t + tau T2_t) + M Y_{t-1} + tau M U_t.
template <typename T, bool TIME>
__global__ __launch_bounds__(GTX* GTX) void k_gen_kkt(int n, int nxi, int nt, const T* __restrict__ x,
                                                      const T* __restrict__ T1, const T* __restrict__ T2,
                                                      T* __restrict__ y, const MemberDev* __restrict__ mem, int shared,
                                                      const int* __restrict__ act, int tiles_x) {
    const int slice = blockIdx.z;
    const int vec = slice / nt, t = slice % nt;
    if (act && !act[vec]) return;
    const int j = blockIdx.y;
    const int ix = (blockIdx.x % tiles_x) * GTX + threadIdx.x % GTX;
    const int iy = (blockIdx.x / tiles_x) * GTX + threadIdx.x / GTX;
    if (ix > n || iy > n) return;
    const int N1 = n + 1;
    const int64_t nodes = (int64_t)N1 * N1;
    const int64_t q = (int64_t)iy * N1 + ix;
    const int64_t tst = (int64_t)nxi * nodes, blk = (int64_t)nt * tst;
    const int64_t cj = (int64_t)t * tst + (int64_t)j * nodes;
    T* RY = y + (int64_t)vec * 3 * blk + cj;
    T* RU = RY + blk;
    T* RL = RU + blk;
    if (ix == 0 || iy == 0 || ix == n || iy == n) {
        RY[q] = RU[q] = RL[q] = T(0);
        return;
    }
    const T* Y = x + (int64_t)vec * 3 * blk + cj;
    const T* U = Y + blk;
    const T* Lm = U + blk;
    const MemberDev md = mem[shared ? 0 : vec];
    const double h = 1.0 / n, w = h * h / 36.0;
    // interior mass stencil; the ring holds no unknowns, its values count as zero
    const bool xl = ix > 1, xr = ix < n - 1, yl = iy > 1, yr = iy < n - 1;
    auto m9 = [&](const T* v) {
        auto g = [&](bool in, int64_t o) { return in ? (double)v[q + o] : 0.0; };
        return w * (16.0 * (double)v[q] + 4.0 * (g(xl, -1) + g(xr, 1) + g(yl, -N1) + g(yr, N1)) +
                    (g(xl && yl, -N1 - 1) + g(xr && yl, -N1 + 1) + g(xl && yr, N1 - 1) + g(xr && yr, N1 + 1)));
    };
    const double hgj = j == 0 ? 1.0 : md.hg;
    const int64_t tj = (int64_t)vec * blk + cj;
    const double t1 = (double)T1[tj + q], t2 = (double)T2[tj + q];
    if (!TIME) {
        RY[q] = (T)(hgj * m9(Y) - t1);
        RU[q] = (T)(md.beta * m9(U) + m9(Lm));
        RL[q] = (T)(-t2 + m9(U));
    } else {
        const double tau = md.tau, Dt = (t == 0 || t == nt - 1) ? 0.5 : 1.0;
        double ry = tau * Dt * hgj * m9(Y) - (m9(Lm) + tau * t1);
        if (t + 1 < nt) ry += m9(Lm + tst);
        double rl = -(m9(Y) + tau * t2) + tau * m9(U);
        if (t > 0) rl += m9(Y - tst);
        RY[q] = (T)ry;
        RU[q] = (T)(md.beta * tau * Dt * m9(U) + tau * m9(Lm));
        RL[q] = (T)rl;
    }
}

}  // namespace

template <typename T>
void launch_gen_sg(const Shape& s, const OpDev& op, bool trunc, const T* X, int64_t xms, int64_t xts, int ilo1,
                   int ihi1, int ilo2, int ihi2, int j0, int L, const T* base, ColMap bmap, T* out, ColMap omap,
                   double scale, int scale_off, double mean_c, int nvec, hipStream_t st) {
    if (L < 1 || nvec < 1) return;
    const int tiles_x = (s.n + 1 + GTX - 1) / GTX;
    const int64_t slices = (int64_t)nvec * s.nt;
    const int chunks = (L + GJC - 1) / GJC;
    if (slices > 65535 || chunks > 65535) throw Error(SG_ERR_INVALID, "general SG apply: launch grid too large");
    hipLaunchKernelGGL(k_gen_sg<T>, dim3(tiles_x * tiles_x, chunks, (unsigned)slices), dim3(GTX * GTX), 0, st, s.n,
                       s.nxi, s.nt, trunc ? op.genBr : op.genB, op.gen_mstride, X, xms, xts, ilo1, ihi1, ilo2, ihi2,
                       j0, L, base, bmap, out, omap, scale, scale_off, mean_c, op.mem, op.mem_shared, op.active,
                       tiles_x);
    SG_HIP(hipGetLastError());
}

template <typename T>
void launch_gen_kkt(const Shape& s, const OpDev& op, const T* x, T* y, T* T1, T* T2, int nvec, hipStream_t st) {
    const int64_t blk = s.blk, tst = s.tstride;
    const ColMap full = [&] {
        ColMap m;
        m.mstride = blk;
        m.tstride = tst;
        m.nodes = s.nodes;
        m.L = s.nxi;
        m.nt = s.nt;
        m.j0 = 0;
        return m;
    }();
    // T1 = A Lambda, T2 = A Y (full operator)
    launch_gen_sg<T>(s, op, false, x + 2 * blk, 3 * blk, tst, 0, s.nxi, 0, 0, 0, s.nxi, (const T*)nullptr, full, T1,
                     full, 1.0, 0, 0.0, nvec, st);
    launch_gen_sg<T>(s, op, false, x, 3 * blk, tst, 0, s.nxi, 0, 0, 0, s.nxi, (const T*)nullptr, full, T2, full, 1.0,
                     0, 0.0, nvec, st);
    const int tiles_x = (s.n + 1 + GTX - 1) / GTX;
    const dim3 grid(tiles_x * tiles_x, s.nxi, (unsigned)((int64_t)nvec * s.nt));
    if (s.time)
        hipLaunchKernelGGL((k_gen_kkt<T, true>), grid, dim3(GTX * GTX), 0, st, s.n, s.nxi, s.nt, x, T1, T2, y, op.mem,
                           op.mem_shared, op.active, tiles_x);
    else
        hipLaunchKernelGGL((k_gen_kkt<T, false>), grid, dim3(GTX * GTX), 0, st, s.n, s.nxi, s.nt, x, T1, T2, y,
                           op.mem, op.mem_shared, op.active, tiles_x);
    SG_HIP(hipGetLastError());
}

template void launch_gen_sg<double>(const Shape&, const OpDev&, bool, const double*, int64_t, int64_t, int, int, int,
                                    int, int, int, const double*, ColMap, double*, ColMap, double, int, double, int,
                                    hipStream_t);
template void launch_gen_sg<float>(const Shape&, const OpDev&, bool, const float*, int64_t, int64_t, int, int, int,
                                   int, int, int, const float*, ColMap, float*, ColMap, double, int, double, int,
                                   hipStream_t);
template void launch_gen_kkt<double>(const Shape&, const OpDev&, const double*, double*, double*, double*, int,
                                     hipStream_t);
template void launch_gen_kkt<float>(const Shape&, const OpDev&, const float*, float*, float*, float*, int,
                                    hipStream_t);

}  // namespace sg
