// Autotuner of the sweep kernels' strip height (node rows per 32-lane strip)
// for the SG operator apply, the hGS off-level right-hand side and the fused
// KKT apply.  Every candidate evaluates the same sums per node in the same
// order, so the choice changes timing only, never results.  Choices are cached
// per process by (device, shape, single member or batch, element type).
#include <array>
#include <map>
#include <mutex>
#include <tuple>

#include "handle.hpp"

namespace sg {
namespace {

using TuneKey = std::tuple<int, int, int, int, int, int, int, int>;   // device n M P nt time B fp32
std::mutex g_tune_mu;
std::map<TuneKey, std::array<int, 3>> g_tune_cache;

float time_launch(hipStream_t st, hipEvent_t e0, hipEvent_t e1, const std::function<void()>& launch) {
    launch();   // warm-up (code object load, caches)
    float best = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
        SG_HIP(hipEventRecord(e0, st));
        launch();
        SG_HIP(hipEventRecord(e1, st));
        SG_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        SG_HIP(hipEventElapsedTime(&ms, e0, e1));
        best = ms < best ? ms : best;
    }
    return best;
}

template <typename T>
std::array<int, 3> tune_type(Handle& h, hipStream_t st) {
    Shape& s = h.s;
    const int B = h.B;
    const bool shared = B == 1;
    const OpDev op = h.op<T>(shared);
    const int64_t N = (int64_t)B * 3 * s.blk;
    // the Krylov work vectors (allocated by every solve anyway) serve as operands
    T* x = reinterpret_cast<T*>(h.ws.get_t<double>("kw", (size_t)N));
    T* y = reinterpret_cast<T*>(h.ws.get_t<double>("kr", (size_t)N));
    SG_HIP(hipMemsetAsync(x, 0, sizeof(T) * N, st));
    hipEvent_t e0, e1;
    SG_HIP(hipEventCreate(&e0));
    SG_HIP(hipEventCreate(&e1));
    std::array<int, 3> best{4, 4, 4};
    try {
        const int d = s.P;   // the widest degree level with its lower neighbour level
        ColMap lm{s.blk, s.tstride, s.nodes, s.off[d + 1] - s.off[d], s.nt, s.off[d]};
        ColMap bm{s.blk, s.tstride, s.nodes, s.nxi, s.nt, 0};
        for (int kind = 0; kind < 3; ++kind) {
            float tbest = 1e30f;
            for (int rows : kSweepRowChoices) {
                s.sweep_rows[sizeof(T) == 4][kind] = rows;
                const float ms = time_launch(st, e0, e1, [&] {
                    if (kind == SWEEP_APPLY)
                        launch_sgx_apply<T>(s, op, x, y, B, 0xffffffffu, st);
                    else if (kind == SWEEP_HGS)
                        launch_sgx_hgs_rhs<T>(s, op, d, h.modes_mask(), 1, 0, x, lm, x, bm, y, lm, B, st);
                    else
                        launch_sgx_kkt<T>(s, op, x, y, B, st);
                });
                if (ms < tbest) {
                    tbest = ms;
                    best[kind] = rows;
                }
            }
            s.sweep_rows[sizeof(T) == 4][kind] = best[kind];
        }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    SG_HIP(hipEventDestroy(e0));
    SG_HIP(hipEventDestroy(e1));
    return best;
}

}  // namespace

void autotune(Handle& h) {
    Shape& s = h.s;
    const int forced = h.opt.sweep_rows;
    for (int t = 0; t < 2; ++t)
        for (int k = 0; k < 3; ++k) s.sweep_rows[t][k] = forced > 0 ? forced : 4;
    if (forced > 0 || s.field != SG_FIELD_AFFINE || s.M > 8) return;      // fixed by the caller, or no sweep kernels for this shape
    const bool need32 = h.opt.precision != SG_PREC_FP64;
    for (int t = 0; t < (need32 ? 2 : 1); ++t) {
        // batches of any size above one share a choice (the serving loop forms
        // batches of every size; a new size should not time the kernels again)
        const TuneKey key{h.device, s.n, s.M, s.P, s.nt, s.time ? 1 : 0, h.B > 1 ? 2 : 1, t};
        std::array<int, 3> rows;
        bool hit = false;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tune_cache.find(key);
            if (it != g_tune_cache.end()) {
                rows = it->second;
                hit = true;
            }
        }
        if (!hit) {
            rows = t == 0 ? tune_type<double>(h, h.stream) : tune_type<float>(h, h.stream);
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tune_cache[key] = rows;
        }
        for (int k = 0; k < 3; ++k) s.sweep_rows[t][k] = rows[k];
    }
}

}  // namespace sg
