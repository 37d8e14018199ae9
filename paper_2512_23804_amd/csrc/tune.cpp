// Autotuner of the sweep kernels' strip height (node rows per 32-lane strip)
// for the SG operator apply, the hGS off-level right-hand side and the fused
// KKT apply.  Every candidate evaluates the same sums per node in the same
// order, so the choice changes timing only, never results.  Choices are cached
// by (device model, shape, single member or batch, element type): in memory
// for the process, and in a text file when the environment variable
// SG_TUNE_CACHE names one (read at the first tuning of the process, rewritten
// after every new choice) or through sg_tune_save / sg_tune_load.
//
// File format: a first line "sgkkt-tune 1", then one entry per line,
//   <arch> <compute units> <n> <M> <P> <n_t> <time> <batch class> <fp32> <apply> <hgs> <kkt>
// with the device's architecture name (no spaces), batch class 1 for one
// member and 2 for more, and the three strip heights in {2, 4, 8}.
#include <array>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>

#include <unistd.h>

#include "handle.hpp"

namespace sg {
namespace {

using TuneKey = std::tuple<std::string, int, int, int, int, int, int, int, int>;   // arch CUs n M P nt time B fp32
using TuneMap = std::map<TuneKey, std::array<int, 3>>;
std::mutex g_tune_mu;
TuneMap g_tune_cache;
bool g_env_loaded = false;
const char* kTuneMagic = "sgkkt-tune 1";

bool valid_rows(int r) { return r == 2 || r == 4 || r == 8; }

// parse a cache file into `out`; strict: the first malformed line is an error
void parse_file(const std::string& path, TuneMap& out) {
    std::ifstream f(path);
    if (!f) throw Error(SG_ERR_INVALID, "tuning cache: cannot open " + path);
    std::string line;
    if (!std::getline(f, line) || line != kTuneMagic)
        throw Error(SG_ERR_INVALID, "tuning cache: " + path + " does not start with '" + kTuneMagic + "'");
    int lineno = 1;
    while (std::getline(f, line)) {
        ++lineno;
        if (line.empty()) continue;
        std::istringstream in(line);
        std::string arch, extra;
        int v[8];
        std::array<int, 3> rows;
        bool ok = static_cast<bool>(in >> arch);
        for (int i = 0; ok && i < 8; ++i) ok = static_cast<bool>(in >> v[i]);
        for (int i = 0; ok && i < 3; ++i) ok = static_cast<bool>(in >> rows[i]) && valid_rows(rows[i]);
        if (ok && (in >> extra)) ok = false;
        if (ok) ok = v[0] > 0 && v[1] >= 8 && v[2] >= 1 && v[3] >= 1 && v[4] >= 1 && (v[5] == 0 || v[5] == 1) &&
                     (v[6] == 1 || v[6] == 2) && (v[7] == 0 || v[7] == 1);
        if (!ok) throw Error(SG_ERR_INVALID, "tuning cache: malformed entry at " + path + ":" + std::to_string(lineno));
        out[TuneKey{arch, v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7]}] = rows;
    }
}

// write the cache atomically (a temporary file named for this process and
// call, then rename); lock held by caller
void write_file(const std::string& path, const TuneMap& m) {
    static unsigned long calls = 0;
    const std::string tmp = path + ".tmp." + std::to_string((long)getpid()) + "." + std::to_string(++calls);
    {
        std::ofstream f(tmp, std::ios::trunc);
        if (!f) throw Error(SG_ERR_INVALID, "tuning cache: cannot write " + tmp);
        f << kTuneMagic << "\n";
        for (const auto& kv : m) {
            const TuneKey& k = kv.first;
            f << std::get<0>(k) << ' ' << std::get<1>(k) << ' ' << std::get<2>(k) << ' ' << std::get<3>(k) << ' '
              << std::get<4>(k) << ' ' << std::get<5>(k) << ' ' << std::get<6>(k) << ' ' << std::get<7>(k) << ' '
              << std::get<8>(k) << ' ' << kv.second[0] << ' ' << kv.second[1] << ' ' << kv.second[2] << "\n";
        }
        if (!f) throw Error(SG_ERR_INVALID, "tuning cache: write to " + tmp + " failed");
    }
    if (std::rename(tmp.c_str(), path.c_str()) != 0) {
        std::remove(tmp.c_str());
        throw Error(SG_ERR_INVALID, "tuning cache: cannot replace " + path);
    }
}

const char* env_path() {
    const char* p = std::getenv("SG_TUNE_CACHE");
    return (p && *p) ? p : nullptr;
}

// first use in the process: merge the file SG_TUNE_CACHE names, if it exists
// (a missing file is an empty cache; a malformed one is reported); lock held
void load_env_once() {
    if (g_env_loaded) return;
    g_env_loaded = true;
    const char* p = env_path();
    if (!p) return;
    std::ifstream probe(p);
    if (!probe) return;
    probe.close();
    TuneMap m;
    parse_file(p, m);
    for (auto& kv : m) g_tune_cache.insert(kv);
}

// "<arch> <CUs>" of a device, the part of the key that a cache file carries
// from one machine to another
std::pair<std::string, int> device_model(int dev) {
    hipDeviceProp_t prop;
    SG_HIP(hipGetDeviceProperties(&prop, dev));
    std::string arch(prop.gcnArchName);
    for (char& c : arch)
        if (c == ' ' || c == '\t') c = '_';
    if (arch.empty()) arch = "unknown";
    return {arch, prop.multiProcessorCount};
}

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
            if (sizeof(T) == 8 && kind == SWEEP_APPLY) continue;   // FP64 SG apply: paired-node kernel, no strip choice
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
    const auto model = device_model(h.device);
    for (int t = 0; t < (need32 ? 2 : 1); ++t) {
        // batches of any size above one share a choice (the serving loop forms
        // batches of every size; a new size should not time the kernels again)
        const TuneKey key{model.first, model.second, s.n, s.M, s.P, s.nt, s.time ? 1 : 0, h.B > 1 ? 2 : 1, t};
        std::array<int, 3> rows;
        bool hit = false;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            load_env_once();
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
            if (const char* p = env_path()) {
                // merge what other processes wrote since this one read the file
                TuneMap disk;
                std::ifstream probe(p);
                if (probe) {
                    probe.close();
                    try {
                        parse_file(p, disk);
                    } catch (const Error&) {
                        disk.clear();      // a file that no longer parses is replaced
                    }
                }
                for (auto& kv : disk) g_tune_cache.insert(kv);
                write_file(p, g_tune_cache);
            }
        }
        for (int k = 0; k < 3; ++k) s.sweep_rows[t][k] = rows[k];
    }
}

void tune_save(const char* path) {
    if (!path || !*path) throw Error(SG_ERR_INVALID, "tuning cache: null or empty path");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_env_once();
    write_file(path, g_tune_cache);
}

void tune_load(const char* path) {
    if (!path || !*path) throw Error(SG_ERR_INVALID, "tuning cache: null or empty path");
    TuneMap m;
    parse_file(path, m);             // nothing is merged unless the whole file parses
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_env_once();
    for (auto& kv : m) g_tune_cache[kv.first] = kv.second;
}

int tune_count() {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_env_once();
    return (int)g_tune_cache.size();
}

void tune_clear() {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_env_loaded = true;             // a cleared cache stays empty until loaded or tuned again
    g_tune_cache.clear();
}

}  // namespace sg
