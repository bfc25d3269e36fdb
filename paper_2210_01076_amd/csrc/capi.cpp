// extern "C" entry points of libqtask.so (declared in include/qtask.h).
// Every entry point catches C++ exceptions and turns them into status codes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>

#include "../../include/qtask.h"
#include "device.h"
#include "lowering.h"
#include "session.h"

using qtask::Session;

struct qtask_s {
    Session *s;
    qtask_s *self;       // guards against stale handles
    bool server_owned;   // owned by a server: queries only
};

namespace qtask {
// used by the server, which owns the sessions it opens
Session *session_of(qtask_t h) { return (h && h->self == h) ? h->s : nullptr; }
void set_server_owned(qtask_t h, bool owned) {
    if (h && h->self == h) h->server_owned = owned;
}
}  // namespace qtask

namespace {

template <typename F>
int guarded(F &&f) {
    try {
        return f();
    } catch (const std::bad_alloc &) {
        return QTASK_E_NOMEM;
    } catch (...) {
        return QTASK_E_ARG;
    }
}

Session *S(qtask_t h) {
    if (!h || h->self != h || !h->s) return nullptr;
    return h->s;
}

// handle for an entry point that changes the circuit or the state
int SM(qtask_t h, Session **s) {
    *s = S(h);
    if (!*s) return QTASK_E_ARG;
    if (h->server_owned) return QTASK_E_BUSY;
    return QTASK_OK;
}

}  // namespace

extern "C" {

const char *qtask_status_string(int status) {
    switch (status) {
    case QTASK_OK: return "ok";
    case QTASK_E_ARG: return "invalid argument";
    case QTASK_E_CONFLICT: return "gate shares a qubit with a gate of the same level";
    case QTASK_E_NOTFOUND: return "unknown level, gate or index";
    case QTASK_E_NOMEM: return "out of device memory or budget";
    case QTASK_E_DEVICE: return "HIP device error";
    case QTASK_E_STALE: return "state is stale: call qtask_update_state first";
    case QTASK_E_UNSUPPORTED: return "unsupported";
    case QTASK_E_BUSY: return "handle busy";
    default: return "unknown status";
    }
}

int qtask_version(int *major, int *minor) {
    if (!major || !minor) return QTASK_E_ARG;
    *major = 1;
    *minor = 0;
    return QTASK_OK;
}

const char *qtask_last_error(qtask_t h) {
    Session *s = S(h);
    if (!s) return "invalid handle";
    return s->last_error.c_str();
}

int qtask_opts_default(qtask_opts *o) {
    if (!o) return QTASK_E_ARG;
    std::memset(o, 0, sizeof(*o));
    o->struct_size = sizeof(*o);
    o->device = 0;
    o->tile_bits = 0;
    o->low_bits = 0;
    o->block_bits = 0;
    o->fusion = QTASK_FUSE_AUTO;
    o->fuse_width = 4;
    o->ckpt_interval = 100;
    o->max_ckpts = -1;
    o->renorm = 1;
    o->autotune = 0;
    o->closed_mode = 1;
    o->relabel = -1;
    return QTASK_OK;
}

int qtask_device_count(int *count) {
    if (!count) return QTASK_E_ARG;
    int c = 0;
    if (hipGetDeviceCount(&c) != hipSuccess) {
        (void)hipGetLastError();
        c = 0;
    }
    *count = c;
    return QTASK_OK;
}

int qtask_create(int n_qubits, qtask_dtype dtype, const qtask_opts *user, qtask_t *out) {
    return guarded([&] {
        if (!out) return QTASK_E_ARG;
        if (n_qubits < 1 || n_qubits > QK_MAX_QUBITS) return QTASK_E_ARG;
        if (dtype != QTASK_C128 && dtype != QTASK_C64) return QTASK_E_ARG;
        qtask_opts o;
        qtask_opts_default(&o);
        if (user) {
            if (user->struct_size < offsetof(qtask_opts, stream) || user->struct_size > sizeof(qtask_opts))
                return QTASK_E_ARG;
            std::memcpy(&o, user, user->struct_size);
            o.struct_size = sizeof(o);
        }
        if (o.tile_bits == 0) o.tile_bits = dtype == QTASK_C128 ? 11 : 12;
        if (o.low_bits == 0) o.low_bits = dtype == QTASK_C128 ? 4 : 5;
        if (o.block_bits == 0) o.block_bits = 10;
        if (o.fuse_width == 0) o.fuse_width = 4;
        if (o.ckpt_interval == 0) o.ckpt_interval = 100;
        if (o.tile_bits < QK_MIN_TILE_BITS || o.tile_bits > QK_MAX_TILE_BITS) return QTASK_E_ARG;
        if (o.low_bits < 0 || o.low_bits > o.tile_bits) return QTASK_E_ARG;
        if (o.block_bits < 0 || o.block_bits > QK_MAX_QUBITS) return QTASK_E_ARG;
        if (o.fusion < QTASK_FUSE_AUTO || o.fusion > QTASK_FUSE_DENSE) return QTASK_E_ARG;
        if (o.fusion == QTASK_FUSE_DENSE && (o.fuse_width < 4 || o.fuse_width > QK_MAX_DENSE_K)) return QTASK_E_ARG;
        if (o.fusion == QTASK_FUSE_DENSE && o.fuse_width > QK_G &&
            std::min(o.tile_bits, std::max(n_qubits, QK_MIN_TILE_BITS)) < 10)
            return QTASK_E_UNSUPPORTED;  // matrix-core stages need tiles of >= 2^10 amplitudes
        if (o.ckpt_interval < 1 || o.max_ckpts < -1) return QTASK_E_ARG;
        if (o.relabel < -1 || o.relabel > 1) return QTASK_E_ARG;
        if (o.ckpt_delta < 0 || o.ckpt_delta > 1) return QTASK_E_ARG;
        if (o.relabel == -1) o.relabel = std::max(n_qubits, QK_MIN_TILE_BITS) >= 26 ? 1 : 0;
        if (o.device < QTASK_DEVICE_NONE) return QTASK_E_ARG;
        if ((o.alloc == nullptr) != (o.free == nullptr)) return QTASK_E_ARG;
        if (o.device >= 0) {
            int count = 0;
            if (hipGetDeviceCount(&count) != hipSuccess) {
                (void)hipGetLastError();
                return QTASK_E_DEVICE;
            }
            if (o.device >= count) return QTASK_E_DEVICE;
        }
        Session *s = new Session(n_qubits, int(dtype), o);
        qtask_s *h = new qtask_s{s, nullptr, false};
        h->self = h;
        *out = h;
        return QTASK_OK;
    });
}

int qtask_destroy(qtask_t h) {
    return guarded([&] {
        Session *s = nullptr;
        if (int rc = SM(h, &s)) return rc;
        delete s;
        h->s = nullptr;
        h->self = nullptr;
        delete h;
        return QTASK_OK;
    });
}

int qtask_insert_level(qtask_t h, qtask_level_t after, qtask_level_t *out) {
    return guarded([&] {
        Session *s = nullptr;
        if (int rc = SM(h, &s)) return rc;
        return s->circ.insert_level(after, out);
    });
}

int qtask_remove_level(qtask_t h, qtask_level_t level) {
    return guarded([&] {
        Session *s = nullptr;
        if (int rc = SM(h, &s)) return rc;
        return s->circ.remove_level(level);
    });
}

int qtask_insert_gate(qtask_t h, qtask_level_t level, qtask_gate_kind kind, const int32_t *qubits, int nq,
                      const double *params, int np, qtask_gate_t *out) {
    return guarded([&] {
        Session *s = nullptr;
        if (int rc = SM(h, &s)) return rc;
        return s->circ.insert_gate(level, int(kind), qubits, nq, params, np, out);
    });
}

int qtask_remove_gate(qtask_t h, qtask_gate_t gate) {
    return guarded([&] {
        Session *s = nullptr;
        if (int rc = SM(h, &s)) return rc;
        return s->circ.remove_gate(gate);
    });
}

int qtask_num_levels(qtask_t h, uint64_t *out) {
    Session *s = S(h);
    if (!s || !out) return QTASK_E_ARG;
    *out = s->circ.num_levels();
    return QTASK_OK;
}

int qtask_level_at(qtask_t h, uint64_t index, qtask_level_t *out) {
    Session *s = S(h);
    if (!s) return QTASK_E_ARG;
    return s->circ.level_at(index, out);
}

int qtask_num_gates(qtask_t h, uint64_t *out) {
    Session *s = S(h);
    if (!s || !out) return QTASK_E_ARG;
    *out = s->circ.num_gates();
    return QTASK_OK;
}

int qtask_update_state(qtask_t h) {
    return guarded([&] {
        Session *s = nullptr;
        if (int rc = SM(h, &s)) return rc;
        return s->update(false);
    });
}


int qtask_update_state_full(qtask_t h) {
    return guarded([&] {
        Session *s = nullptr;
        if (int rc = SM(h, &s)) return rc;
        return s->update(true);
    });
}

int qtask_last_update_stats(qtask_t h, qtask_stats *out) {
    Session *s = S(h);
    if (!s || !out) return QTASK_E_ARG;
    *out = s->last;
    return QTASK_OK;
}

int qtask_read_amplitudes(qtask_t h, uint64_t first, uint64_t count, void *host_out) {
    return guarded([&] {
        Session *s = S(h);
        if (!s) return QTASK_E_ARG;
        return s->read(first, count, host_out);
    });
}

int qtask_norm(qtask_t h, double *out) {
    return guarded([&] {
        Session *s = S(h);
        if (!s || !out) return QTASK_E_ARG;
        return s->norm(out);
    });
}

int qtask_inner(qtask_t a, qtask_t b, double re_im[2]) {
    return guarded([&] {
        Session *x = S(a), *y = S(b);
        if (!x || !y || !re_im) return QTASK_E_ARG;
        if (x->n != y->n) return QTASK_E_ARG;
        if (x->plan_only || y->plan_only) return QTASK_E_UNSUPPORTED;
        if (x->opts.device != y->opts.device) return QTASK_E_ARG;
        if (!x->state_valid() || !y->state_valid() || x->circ.edited() || y->circ.edited()) return QTASK_E_STALE;
        if (hipSetDevice(x->opts.device) != hipSuccess) return QTASK_E_DEVICE;
        const uint64_t N = uint64_t(1) << x->n_int;
        const uint32_t g = qtask::reduce_grid(N);
        double *tmp = static_cast<double *>(x->dalloc((2 * size_t(g) + 2) * sizeof(double)));
        if (!tmp) return QTASK_E_NOMEM;
        if (hipStreamSynchronize(y->stream) != hipSuccess) { x->dfree(tmp); return QTASK_E_DEVICE; }
        int rc = QTASK_OK;
        double v[2] = {0, 0};
        if (qtask::launch_inner(x->dtype, y->dtype, x->state(), y->state(), N, tmp + 2, tmp, x->stream) != hipSuccess ||
            hipMemcpyAsync(v, tmp, sizeof(v), hipMemcpyDeviceToHost, x->stream) != hipSuccess ||
            hipStreamSynchronize(x->stream) != hipSuccess)
            rc = QTASK_E_DEVICE;
        x->dfree(tmp);
        if (rc == QTASK_OK) { re_im[0] = v[0]; re_im[1] = v[1]; }
        return rc;
    });
}

int qtask_inner_noalloc(qtask_t a, qtask_t b, double re_im[2]) {
    return guarded([&] {
        Session *x = S(a), *y = S(b);
        if (!x || !y || !re_im) return QTASK_E_ARG;
        if (x->n != y->n) return QTASK_E_ARG;
        if (x->plan_only || y->plan_only) return QTASK_E_UNSUPPORTED;
        if (x->opts.device != y->opts.device) return QTASK_E_ARG;
        if (!x->state_valid() || !y->state_valid() || x->circ.edited() || y->circ.edited()) return QTASK_E_STALE;
        if (hipSetDevice(x->opts.device) != hipSuccess) return QTASK_E_DEVICE;
        const uint64_t N = uint64_t(1) << x->n_int;
        const uint32_t g = qtask::reduce_grid(N);
        double *scr = nullptr;
        size_t cap = 0;
        if (qtask::noalloc_scratch(x->opts.device, &scr, &cap) != hipSuccess) return QTASK_E_DEVICE;
        if (2 * size_t(g) + 2 > cap) {
            x->last_error = "qtask_inner_noalloc: the reduction needs more partial sums than the fixed scratch holds";
            return QTASK_E_UNSUPPORTED;
        }
        if (hipStreamSynchronize(y->stream) != hipSuccess) return QTASK_E_DEVICE;
        double v[2] = {0, 0};
        if (qtask::launch_inner(x->dtype, y->dtype, x->state(), y->state(), N, scr + 2, scr, x->stream) != hipSuccess ||
            hipMemcpyAsync(v, scr, sizeof(v), hipMemcpyDeviceToHost, x->stream) != hipSuccess ||
            hipStreamSynchronize(x->stream) != hipSuccess)
            return QTASK_E_DEVICE;
        re_im[0] = v[0];
        re_im[1] = v[1];
        return QTASK_OK;
    });
}

int qtask_compare_states(qtask_t a, qtask_t b, uint64_t *n_diff) {
    return guarded([&] {
        Session *x = S(a), *y = S(b);
        if (!x || !y || !n_diff) return QTASK_E_ARG;
        if (x->n != y->n || x->dtype != y->dtype || x->opts.device != y->opts.device) return QTASK_E_ARG;
        if (x->plan_only || y->plan_only) return QTASK_E_UNSUPPORTED;
        if (!x->state_valid() || !y->state_valid() || x->circ.edited() || y->circ.edited()) return QTASK_E_STALE;
        if (hipSetDevice(x->opts.device) != hipSuccess) return QTASK_E_DEVICE;
        const uint64_t N = uint64_t(1) << x->n_int;
        const uint32_t g = qtask::reduce_grid(N);
        auto *tmp = static_cast<unsigned long long *>(x->dalloc((size_t(g) + 1) * sizeof(unsigned long long)));
        if (!tmp) return QTASK_E_NOMEM;
        if (hipStreamSynchronize(y->stream) != hipSuccess) { x->dfree(tmp); return QTASK_E_DEVICE; }
        int rc = QTASK_OK;
        unsigned long long v = 0;
        if (qtask::launch_compare(x->dtype, x->state(), y->state(), N, tmp + 1, tmp, x->stream) != hipSuccess ||
            hipMemcpyAsync(&v, tmp, sizeof(v), hipMemcpyDeviceToHost, x->stream) != hipSuccess ||
            hipStreamSynchronize(x->stream) != hipSuccess)
            rc = QTASK_E_DEVICE;
        x->dfree(tmp);
        if (rc == QTASK_OK) *n_diff = v;
        return rc;
    });
}

int qtask_state_hash(qtask_t h, uint64_t *out) {
    return guarded([&] {
        Session *s = S(h);
        if (!s || !out) return QTASK_E_ARG;
        return s->hash(out);
    });
}

int qtask_state_device_ptr(qtask_t h, const void **ptr, uint64_t *bytes) {
    Session *s = S(h);
    if (!s || !ptr || !bytes) return QTASK_E_ARG;
    if (s->plan_only) return QTASK_E_UNSUPPORTED;
    if (!s->state_valid() || s->circ.edited()) return QTASK_E_STALE;
    *ptr = s->state();
    *bytes = s->state_bytes();
    return QTASK_OK;
}

int qtask_device_bytes(qtask_t h, uint64_t *out) {
    Session *s = S(h);
    if (!s || !out) return QTASK_E_ARG;
    *out = s->device_bytes();
    return QTASK_OK;
}

int qtask_get_opts(qtask_t h, qtask_opts *out) {
    Session *s = S(h);
    if (!s || !out) return QTASK_E_ARG;
    *out = s->opts;
    return QTASK_OK;
}

int qtask_dump_plan(qtask_t h, const char *path) {
    return guarded([&] {
        Session *s = S(h);
        if (!s || !path) return QTASK_E_ARG;
        return s->dump(path);
    });
}

int qtask_copy_bandwidth(int device, uint64_t bytes, int iters, double *gbps) {
    return guarded([&] {
        if (!gbps || iters < 1 || bytes < 256) return QTASK_E_ARG;
        if (hipSetDevice(device) != hipSuccess) return QTASK_E_DEVICE;
        bytes &= ~uint64_t(255);
        void *a = nullptr, *b = nullptr;
        if (hipMalloc(&a, bytes) != hipSuccess) { (void)hipGetLastError(); return QTASK_E_NOMEM; }
        if (hipMalloc(&b, bytes) != hipSuccess) { (void)hipGetLastError(); (void)hipFree(a); return QTASK_E_NOMEM; }
        int rc = QTASK_OK;
        hipStream_t s = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        float ms = 0;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
            hipEventCreate(&e1) != hipSuccess || hipMemsetAsync(a, 0, bytes, s) != hipSuccess ||
            qtask::launch_copy(b, a, bytes / 32, s) != hipSuccess || hipEventRecord(e0, s) != hipSuccess)
            rc = QTASK_E_DEVICE;
        for (int i = 0; i < iters && rc == QTASK_OK; ++i)
            if (qtask::launch_copy((i & 1) ? a : b, (i & 1) ? b : a, bytes / 32, s) != hipSuccess) rc = QTASK_E_DEVICE;
        if (rc == QTASK_OK && (hipEventRecord(e1, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess ||
                               hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            rc = QTASK_E_DEVICE;
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (s) (void)hipStreamDestroy(s);
        (void)hipFree(a);
        (void)hipFree(b);
        if (rc == QTASK_OK) *gbps = 2.0 * double(bytes) * iters / (double(ms) * 1e-3) / 1e9;
        return rc;
    });
}

}  // extern "C"
