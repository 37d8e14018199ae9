// extern "C" entry points declared in include/sg.h.  Every call converts C++
// exceptions into status codes and a thread-local message.
#include <cstring>
#include <string>

#include "handle.hpp"

struct sg_handle {
    std::unique_ptr<sg::Handle> h;
};

namespace {
thread_local std::string g_last_error;
}  // namespace

namespace sg {
void set_last_error(const std::string& msg) { g_last_error = msg; }
}  // namespace sg

namespace {

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

template <typename F>
int guarded(F&& f) {
    try {
        g_last_error.clear();
        return f();
    } catch (const sg::Error& e) {
        return fail(e.code, e.what());
    } catch (const std::bad_alloc&) {
        return fail(SG_ERR_NOMEM, "host allocation failed");
    } catch (const std::exception& e) {
        return fail(SG_ERR_INVALID, e.what());
    } catch (...) {
        return fail(SG_ERR_INVALID, "unknown failure");
    }
}

int check_vec_args(const sg_handle* h, const void* a, const void* b, int32_t nvec, int32_t dtype) {
    if (!h || !h->h) return fail(SG_ERR_INVALID, "null handle");
    if (!a || !b) return fail(SG_ERR_INVALID, "null vector pointer");
    if (dtype != SG_FP64 && dtype != SG_FP32) return fail(SG_ERR_INVALID, "dtype must be SG_FP64 or SG_FP32");
    if (nvec < 1) return fail(SG_ERR_INVALID, "nvec must be >= 1");
    if (h->h->B > 1 && nvec != h->h->B) return fail(SG_ERR_INVALID, "nvec must equal the number of members");
    if ((int64_t)nvec * h->h->s.nt > 65535) return fail(SG_ERR_INVALID, "nvec * n_t above 65535");
    return SG_OK;
}

}  // namespace

extern "C" {

void sg_default_options(sg_options* opt) {
    if (opt) sg::default_options(opt);
}

int sg_validate(const sg_problem* prob, const sg_options* opt) {
    return guarded([&] {
        sg::validate(prob, 1, opt);
        return SG_OK;
    });
}

int sg_setup(const sg_problem* probs, int32_t count, const sg_options* opt, void* stream, sg_handle** out) {
    return guarded([&] {
        if (!out) return fail(SG_ERR_INVALID, "out is NULL");
        *out = nullptr;
        sg::validate(probs, count, opt);   // host-only checks before any device work
        auto h = sg::build_handle(probs, count, opt, (hipStream_t)stream);
        *out = new sg_handle{std::move(h)};
        return SG_OK;
    });
}

int sg_query(const sg_handle* h, sg_sizes* out) {
    return guarded([&] {
        if (!h || !h->h || !out) return fail(SG_ERR_INVALID, "null argument");
        const sg::Shape& s = h->h->s;
        std::memset(out, 0, sizeof(*out));
        out->n = s.n;
        out->M = s.M;
        out->P = s.P;
        out->n_t = s.nt;
        out->n_xi = s.nxi;
        out->members = h->h->B;
        out->nodes = s.nodes;
        out->block_elems = s.blk;
        out->kkt_elems = 3 * s.blk;
        for (int d = 0; d <= s.P + 1 && d < 17; ++d) out->level_offsets[d] = s.off[d];
        for (int t = 0; t < 2; ++t)
            for (int k = 0; k < 3; ++k) out->sweep_rows[t][k] = s.sweep_rows[t][k];
        return SG_OK;
    });
}

int sg_get_multiindex(const sg_handle* h, int32_t* out) {
    return guarded([&] {
        if (!h || !h->h || !out) return fail(SG_ERR_INVALID, "null argument");
        std::memcpy(out, h->h->ht.alpha.data(), h->h->ht.alpha.size() * sizeof(int32_t));
        return SG_OK;
    });
}

int sg_get_gtable(const sg_handle* h, int32_t* idx, double* val) {
    return guarded([&] {
        if (!h || !h->h || !idx || !val) return fail(SG_ERR_INVALID, "null argument");
        std::memcpy(idx, h->h->ht.nbr_idx.data(), h->h->ht.nbr_idx.size() * sizeof(int32_t));
        std::memcpy(val, h->h->ht.nbr_val.data(), h->h->ht.nbr_val.size() * sizeof(double));
        return SG_OK;
    });
}

int sg_get_rhs(sg_handle* h, double* b_dev) {
    return guarded([&] {
        if (!h || !h->h || !b_dev) return fail(SG_ERR_INVALID, "null argument");
        sg::Handle& H = *h->h;
        SG_HIP(hipMemcpyAsync(b_dev, H.d_rhs, sizeof(double) * H.B * 3 * H.s.blk, hipMemcpyDeviceToDevice, H.stream));
        SG_HIP(hipStreamSynchronize(H.stream));
        return SG_OK;
    });
}

int sg_apply_operator(sg_handle* h, const void* x_dev, void* y_dev, int32_t nvec, int32_t dtype, void* stream) {
    return guarded([&] {
        int rc = check_vec_args(h, x_dev, y_dev, nvec, dtype);
        if (rc) return rc;
        sg::Handle& H = *h->h;
        hipStream_t st = stream ? (hipStream_t)stream : H.stream;
        if (dtype == SG_FP64)
            sg::operator_apply<double>(H, (const double*)x_dev, (double*)y_dev, nvec, H.B == 1, st);
        else
            sg::operator_apply<float>(H, (const float*)x_dev, (float*)y_dev, nvec, H.B == 1, st);
        return SG_OK;
    });
}

int sg_apply_kkt(sg_handle* h, const void* x_dev, void* y_dev, int32_t nvec, int32_t dtype, void* stream) {
    return guarded([&] {
        int rc = check_vec_args(h, x_dev, y_dev, nvec, dtype);
        if (rc) return rc;
        sg::Handle& H = *h->h;
        hipStream_t st = stream ? (hipStream_t)stream : H.stream;
        if (dtype == SG_FP64)
            sg::kkt_apply<double>(H, (const double*)x_dev, (double*)y_dev, nvec, H.B == 1, st);
        else
            sg::kkt_apply<float>(H, (const float*)x_dev, (float*)y_dev, nvec, H.B == 1, st);
        return SG_OK;
    });
}

int sg_precond_apply(sg_handle* h, const void* r_dev, void* z_dev, int32_t nvec, int32_t dtype, void* stream) {
    return guarded([&] {
        int rc = check_vec_args(h, r_dev, z_dev, nvec, dtype);
        if (rc) return rc;
        sg::Handle& H = *h->h;
        hipStream_t st = stream ? (hipStream_t)stream : H.stream;
        if (dtype == SG_FP64)
            sg::precond_apply<double>(H, (const double*)r_dev, (double*)z_dev, nvec, H.B == 1, st);
        else
            sg::precond_apply<float>(H, (const float*)r_dev, (float*)z_dev, nvec, H.B == 1, st);
        return SG_OK;
    });
}

int sg_precond_apply_noalloc(sg_handle* h, const void* r_dev, void* z_dev, int32_t nvec, int32_t dtype,
                             void* stream) {
    return guarded([&] {
        int rc = check_vec_args(h, r_dev, z_dev, nvec, dtype);
        if (rc) return rc;
        sg::Handle& H = *h->h;
        int dev = -1;
        SG_HIP(hipGetDevice(&dev));
        if (dev != H.device) return fail(SG_ERR_INVALID, "the handle's device must be current");
        void* base = sg::noalloc_scratch(dev);
        hipStream_t st = stream ? (hipStream_t)stream : H.stream;
        struct ArenaGuard {
            sg::Workspace& ws;
            ~ArenaGuard() { ws.end_arena(); }
        } guard{H.ws};
        H.ws.begin_arena(base, sg::noalloc_scratch_bytes());
        // every scratch buffer is carved before the first launch: a call that
        // does not fit fails here with SG_ERR_NOMEM and launches nothing
        if (dtype == SG_FP64) {
            sg::precond_reserve<double>(H, nvec);
            sg::precond_apply<double>(H, (const double*)r_dev, (double*)z_dev, nvec, H.B == 1, st);
        } else {
            sg::precond_reserve<float>(H, nvec);
            sg::precond_apply<float>(H, (const float*)r_dev, (float*)z_dev, nvec, H.B == 1, st);
        }
        return SG_OK;
    });
}

int sg_solve(sg_handle* h, const double* b_dev, double* x_dev, sg_solve_info* info) {
    return guarded([&] {
        if (!h || !h->h || !x_dev) return fail(SG_ERR_INVALID, "null argument");
        return sg::solve(*h->h, b_dev, x_dev, info);
    });
}

void sg_destroy(sg_handle* h) {
    if (!h) return;
    try {
        if (h->h) (void)hipStreamSynchronize(h->h->stream);
        delete h;
    } catch (...) {
    }
}

int sg_tune_save(const char* path) {
    return guarded([&] {
        sg::tune_save(path);
        return SG_OK;
    });
}

int sg_tune_load(const char* path) {
    return guarded([&] {
        sg::tune_load(path);
        return SG_OK;
    });
}

int sg_tune_count(void) {
    return guarded([&] { return sg::tune_count(); });
}

int sg_tune_clear(void) {
    return guarded([&] {
        sg::tune_clear();
        return SG_OK;
    });
}

const char* sg_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
