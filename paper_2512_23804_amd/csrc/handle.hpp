// Handle: one batch of same-shape problems and its device state.
#pragma once

#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"

namespace sg {

// Device blocks kept for reuse instead of being freed.  The server builds and
// releases a handle per batch; hipFree synchronises the whole device, so its
// handles take their memory from one pool that frees nothing until it is
// trimmed (on an allocation failure, or when the server is destroyed).  A
// request is served by the smallest cached block that is at least as large
// and at most 25% (or 8 MiB) larger; blocks are handed out only by the thread
// whose stream has finished with them (a handle releases its memory after its
// stream synchronised).
class DevicePool {
  public:
    ~DevicePool() { trim(); }
    void* alloc(size_t bytes) {
        bytes = (bytes + 255) / 256 * 256;
        {
            std::lock_guard<std::mutex> lk(mu_);
            auto it = free_.lower_bound(bytes);
            if (it != free_.end() && it->first <= bytes + std::max<size_t>(bytes / 4, size_t(8) << 20)) {
                void* p = it->second;
                cached_ -= it->first;
                free_.erase(it);
                return p;
            }
        }
        void* p = nullptr;
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            trim();
            e = hipMalloc(&p, bytes);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                throw Error(SG_ERR_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed: " +
                                              hipGetErrorString(e));
            }
        }
        std::lock_guard<std::mutex> lk(mu_);
        size_of_[p] = bytes;
        return p;
    }
    void release(void* p) {
        if (!p) return;
        std::lock_guard<std::mutex> lk(mu_);
        auto it = size_of_.find(p);
        if (it == size_of_.end()) return;
        free_.emplace(it->second, p);
        cached_ += it->second;
    }
    void trim() {
        std::lock_guard<std::mutex> lk(mu_);
        for (auto& kv : free_) {
            (void)hipFree(kv.second);
            size_of_.erase(kv.second);
        }
        free_.clear();
        cached_ = 0;
    }
    size_t cached() const { return cached_; }

  private:
    std::mutex mu_;
    std::multimap<size_t, void*> free_;
    std::map<void*, size_t> size_of_;
    size_t cached_ = 0;
};

// Grow-only named device buffers owned by a handle.  While an arena is set
// (begin_arena), named buffers are carved from that caller-provided device
// memory instead (256-byte aligned, same name -> same buffer for the arena's
// lifetime) and nothing is allocated; a request beyond the arena's capacity
// throws SG_ERR_NOMEM.
class Workspace {
  public:
    ~Workspace() { release(); }
    void set_pool(DevicePool* pool) { pool_ = pool; }
    void begin_arena(void* base, size_t cap) {
        arena_ = static_cast<char*>(base);
        arena_cap_ = cap;
        arena_used_ = 0;
        arena_bufs_.clear();
    }
    void end_arena() {
        arena_ = nullptr;
        arena_cap_ = arena_used_ = 0;
        arena_bufs_.clear();
    }
    bool in_arena() const { return arena_ != nullptr; }
    void* get(const std::string& name, size_t bytes) {
        if (arena_) return carve(name, bytes);
        auto it = bufs_.find(name);
        if (it != bufs_.end() && it->second.second >= bytes) return it->second.first;
        if (it != bufs_.end()) {
            free_block(it->second.first);
            bufs_.erase(it);
        }
        void* p = nullptr;
        if (pool_) {
            p = pool_->alloc(bytes < 256 ? 256 : bytes);
        } else {
            hipError_t e = hipMalloc(&p, bytes < 256 ? 256 : bytes);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                throw Error(SG_ERR_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes for '" + name +
                                              "' failed: " + hipGetErrorString(e));
            }
        }
        bufs_[name] = {p, bytes};
        total_ += bytes;
        ++gen_;
        return p;
    }
    template <typename T>
    T* get_t(const std::string& name, size_t count) {
        return static_cast<T*>(get(name, count * sizeof(T)));
    }
    void release() {
        for (auto& kv : bufs_) free_block(kv.second.first);
        bufs_.clear();
        total_ = 0;
    }
    size_t total() const { return total_; }
    uint64_t generation() const { return gen_; }   // changes whenever a buffer is (re)allocated

  private:
    void free_block(void* p) {
        if (pool_)
            pool_->release(p);
        else
            (void)hipFree(p);
    }
    void* carve(const std::string& name, size_t bytes) {
        auto it = arena_bufs_.find(name);
        if (it != arena_bufs_.end() && it->second.second >= bytes) return it->second.first;
        const size_t start = (arena_used_ + 255) / 256 * 256;
        if (start > arena_cap_ || bytes > arena_cap_ - start)
            throw Error(SG_ERR_NOMEM, "scratch of " + std::to_string(start + bytes) + " bytes needed ('" + name +
                                          "'), above the fixed maximum of " + std::to_string(arena_cap_) + " bytes");
        void* p = arena_ + start;
        arena_used_ = start + bytes;
        arena_bufs_[name] = {p, bytes};
        return p;
    }
    std::map<std::string, std::pair<void*, size_t>> bufs_;
    size_t total_ = 0;
    uint64_t gen_ = 0;
    char* arena_ = nullptr;
    size_t arena_cap_ = 0, arena_used_ = 0;
    DevicePool* pool_ = nullptr;
    std::map<std::string, std::pair<void*, size_t>> arena_bufs_;
};

// HIP-event timing of one kernel's launches (sg_options.profile).
struct Prof {
    int kind = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    size_t used = 0;
    double bytes = 0.0;
    void reset() {
        used = 0;
        bytes = 0.0;
    }
    ~Prof() {
        for (auto& e : ev) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
    }
};

// Instantiated graphs of one FGMRES iteration, keyed by (restart position j,
// precision variant: bit 0 FP32 preconditioner, bit 1 FP32 operator, bit 2
// FP32 basis), valid for one workspace generation.
struct GraphCache {
    std::map<std::pair<int, int>, hipGraphExec_t> exec;
    uint64_t gen = ~0ull;
    bool warm[8] = {false, false, false, false, false, false, false, false};
    void clear() {
        for (auto& kv : exec) (void)hipGraphExecDestroy(kv.second);
        exec.clear();
        for (bool& w : warm) w = false;
    }
    ~GraphCache() { clear(); }
};

struct Handle {
    Shape s{};
    int B = 1;                          // members
    int mg_tail_max = 64;               // finest multigrid level run by the fused single-workgroup tail
    sg_options opt{};
    hipStream_t stream = nullptr;
    int device = 0;
    double t_setup_ms = 0.0;
    DevicePool* pool = nullptr;         // device memory source (nullptr: hipMalloc / hipFree)

    HostTables ht;
    std::vector<MemberDev> mem_host;
    std::vector<LevelDev> lev_host;     // [member][kMaxLevels]
    std::vector<double> coef_host;      // [member][M+1][n][n]
    std::vector<double> ainv_host;      // [member][64][64]
    // nonzero chaos columns of the right-hand sides: [member][2][nt][nodes]
    // (state block, column 0, every t; adjoint block, column 0, every t);
    // every other entry of a KKT right-hand side is zero
    std::vector<double> rhs_host;

    // device-resident constant data
    int32_t* d_nbr_idx = nullptr;
    double* d_nbr_val = nullptr;
    double* d_coef64 = nullptr;
    float* d_coef32 = nullptr;
    MemberDev* d_mem = nullptr;
    LevelDev* d_lev = nullptr;
    double* d_ainv64 = nullptr;
    float* d_ainv32 = nullptr;
    double* d_rhs = nullptr;
    double* d_dst = nullptr;            // sine-transform tables: [2n] sin(pi m / n), [n+1] k_p, [n+1] m_p
    double* d_genB = nullptr;           // general coupling: [member][e][i][j] B_e over all terms
    double* d_genBr = nullptr;          // the same over the terms l < truncation r (null when r = n_A)

    Workspace ws;
    Prof prof;
    GraphCache graphs;
    double* h_pinned = nullptr;        // host-pinned scratch for small readbacks and uploads
    size_t h_pinned_count = 0;
    // per-vector activity flags the operator and preconditioner kernels honour
    // (set by FGMRES around its iterations; null: every vector is processed)
    const int* active = nullptr;

    // coefficient terms kept by the hGS truncation (Section 5's n_tau)
    int trunc_r() const {
        const int nA = s.field == SG_FIELD_LOGNORMAL ? s.nA : s.M + 1;
        return opt.truncation_r <= 0 ? nA : opt.truncation_r;
    }
    uint32_t modes_mask() const {
        // log-normal field: 0 mean-based, all ones every term, else the truncated terms (genBr)
        if (s.field == SG_FIELD_LOGNORMAL) return trunc_r() <= 1 ? 0u : trunc_r() < s.nA ? 0x7fffffffu : 0xffffffffu;
        const int r = opt.truncation_r <= 0 ? s.M + 1 : opt.truncation_r;
        uint32_t m = 0;
        for (int k = 1; k < r && k <= s.M; ++k) m |= 1u << (k - 1);
        return m;
    }
    template <typename T>
    OpDev op(bool shared) const {
        OpDev o;
        o.nbr_idx = d_nbr_idx;
        o.nbr_val = d_nbr_val;
        o.coef = sizeof(T) == 8 ? (const void*)d_coef64 : (const void*)d_coef32;
        o.coef64 = d_coef64;
        o.coef_mstride = shared ? 0 : (int64_t)(s.M + 1) * s.n * s.n;
        o.mem = d_mem;
        o.mem_shared = shared ? 1 : 0;
        o.active = active;
        o.genB = d_genB;
        o.genBr = d_genBr ? d_genBr : d_genB;
        o.gen_mstride = shared ? 0 : (int64_t)s.n * s.n * s.nxi * s.nxi;
        o.gen = s.field == SG_FIELD_LOGNORMAL ? 1 : 0;
        o.off_sign = 1.0;
        return o;
    }
    template <typename T>
    const T* ainv() const {
        return sizeof(T) == 8 ? (const T*)(const void*)d_ainv64 : (const T*)(const void*)d_ainv32;
    }
    ~Handle();
};

// abi.cpp: message returned by sg_last_error() on this thread
void set_last_error(const std::string& msg);

// setup.cpp
void default_options(sg_options* o);
void validate(const sg_problem* probs, int count, const sg_options* opt);   // throws Error
void autotune(Handle& h);   // tune.cpp: strip heights of the sweep kernels (sg_options.sweep_rows)
void tune_save(const char* path);   // tune.cpp: the strip-height cache as a text file
void tune_load(const char* path);
int tune_count();
void tune_clear();
std::unique_ptr<Handle> build_handle(const sg_problem* probs, int count, const sg_options* opt, hipStream_t st,
                                     DevicePool* pool = nullptr);
// Replace member b's problem (same n, M, P, n_t and options as the handle):
// its coefficient modes, scalars, multigrid constants, coarse inverse and
// right-hand side, on the handle's stream (returns after the copies).
void set_member(Handle& h, int b, const sg_problem& p);
// lognormal.cpp: Hermite triple-product matrices H [n_A][nxi][nxi] and the
// per-element chaos coefficients kappa [n_A][n][n] of the log-normal field,
// and the element couplings B_e = sum_{l < r} kappa_l(e) H_l ([e][i][j])
void lognormal_tables(const sg_problem& p, int nxi, const std::vector<int32_t>& alpha, std::vector<double>& H,
                      std::vector<double>& kappa, int& nA);
void lognormal_element_matrices(int n, int nxi, int nA, int r, const std::vector<double>& H,
                                const std::vector<double>& kappa, double* B);
std::vector<int32_t> multi_indices(int M, int P);
int binom(int n, int k);

// solver.cpp
bool prof_begin(Handle& h, int kind, hipStream_t st);        // true if this launch is timed
void prof_end(Handle& h, hipStream_t st, double bytes);
double prof_collect_ms(Handle& h);                           // waits for the events, sums durations
template <typename T>
void precond_apply(Handle& h, const T* r, T* z, int nvec, bool shared, hipStream_t st);
template <typename T>
void precond_reserve(Handle& h, int nvec);                   // request precond_apply's scratch up front
template <typename T>
void kkt_apply(Handle& h, const T* x, T* y, int nvec, bool shared, hipStream_t st);

// noalloc.hip: the library's fixed device scratch array (for the entry point
// that allocates nothing): its address on `device` (resolved once per device,
// with that device current) and its size in bytes
void* noalloc_scratch(int device);
size_t noalloc_scratch_bytes();
template <typename T>
void operator_apply(Handle& h, const T* x, T* y, int nvec, bool shared, hipStream_t st);
// Source of problems for the member slots of a running solve (serving).  At
// every restart boundary the solve reports each member whose solve has ended
// (done) and then asks for a problem for every free slot (next); a slot
// filled there starts from x = 0 with the problem's own right-hand side, so
// its arithmetic is that of an alone solve.
struct SlotFeed {
    virtual ~SlotFeed() = default;
    // slot q ended: its FP64 solution is x_member (device, one KKT vector,
    // valid until the slot is refilled), its report info
    virtual void done(int q, const double* x_member, const sg_solve_info& info, hipStream_t st) = 0;
    // a problem for free slot q, of the handle's shape and options (its arrays
    // stay valid until done(q) reports it), or false
    virtual bool next(int q, sg_problem& p) = 0;
};
// b_dev null: the handle's own right-hand sides.  With a feed, x_dev is the
// batch's working solution and the members' results go through the feed;
// info may then be null.
int solve(Handle& h, const double* b_dev, double* x_dev, sg_solve_info* info, SlotFeed* feed = nullptr);

}  // namespace sg
