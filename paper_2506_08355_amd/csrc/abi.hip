// C ABI of the library (declared in include/lrep.h): contexts, operators,
// blocking solves and the request queue of the serving interface.
#include <algorithm>
#include <chrono>
#include <cstring>

#include "internal.hpp"

using namespace lrep;

struct lrep_ctx_s : public Ctx {};
struct lrep_op_s : public Op {};

namespace lrep {

thread_local Reservation* t_reservation = nullptr;
thread_local bool t_serving = false;

DevBuf::~DevBuf() { release(); }

int DevBuf::alloc(Ctx* c, size_t nbytes) {
    release();
    ctx = c;
    if (nbytes == 0) nbytes = 8;
    Reservation* rv = t_reservation;
    if (rv && rv->ctx == c && rv->left >= nbytes) {
        // already charged at admission
        void* q = nullptr;
        hipError_t e = hipMalloc(&q, nbytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return e == hipErrorOutOfMemory ? LREP_ENOMEM : LREP_EDEVICE;
        }
        rv->left -= nbytes;
        p = static_cast<double*>(q);
        bytes = nbytes;
        return LREP_OK;
    }
    if (c->budget) {
        size_t cur = c->used.load();
        do {
            if (cur + nbytes > c->budget) return LREP_ENOMEM;
        } while (!c->used.compare_exchange_weak(cur, cur + nbytes));
    } else {
        c->used += nbytes;
    }
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, nbytes);
    if (e != hipSuccess) {
        c->used -= nbytes;
        (void)hipGetLastError();
        return e == hipErrorOutOfMemory ? LREP_ENOMEM : LREP_EDEVICE;
    }
    p = static_cast<double*>(q);
    bytes = nbytes;
    return LREP_OK;
}

void DevBuf::release() {
    if (p) {
        (void)hipFree(p);
        ctx->used -= bytes;
    }
    p = nullptr;
    bytes = 0;
}

}  // namespace lrep

namespace {

int set_device(Ctx* c) {
    return hipSetDevice(c->device) == hipSuccess ? LREP_OK : LREP_EDEVICE;
}

// Serving worker: takes queued requests in arrival order, skipping those
// whose footprint does not fit the free budget now (a later, smaller one may),
// reserves the footprint and runs the solve on its own stream.  A request
// that could not fit even with no other request running fails at once with
// LREP_ENOMEM.
void worker_main(Ctx* c) {
    (void)hipSetDevice(c->device);
    hipStream_t st = nullptr;
    const bool ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
    std::unique_lock<std::mutex> lk(c->q_mu);
    if (!ok) {
        // no stream: fail what is queued now and refuse later submissions
        c->broken = true;
        for (uint64_t id : c->queue) {
            auto it = c->tickets.find(id);
            if (it != c->tickets.end() && it->second.state == 0) {
                it->second.state = 2;
                it->second.rc = LREP_EDEVICE;
            }
        }
        c->queue.clear();
        c->q_cv.notify_all();
        return;
    }
    for (;;) {
        uint64_t id = 0;
        size_t fp = 0;
        for (;;) {
            if (c->stopping && c->queue.empty()) break;
            const size_t used = c->used.load();
            const size_t base = used >= c->reserved ? used - c->reserved : 0;
            for (auto q = c->queue.begin(); q != c->queue.end();) {
                auto it = c->tickets.find(*q);
                if (it == c->tickets.end() || it->second.state != 0) {
                    q = c->queue.erase(q);
                    continue;
                }
                const size_t f = it->second.footprint;
                if (c->budget && base + f > c->budget) {
                    // cannot fit even alone
                    it->second.state = 2;
                    it->second.rc = LREP_ENOMEM;
                    q = c->queue.erase(q);
                    c->q_cv.notify_all();
                    continue;
                }
                if (!c->budget || used + f <= c->budget) {
                    id = *q;
                    fp = f;
                    c->queue.erase(q);
                    break;
                }
                ++q;
            }
            if (id || c->stopping) break;
            c->q_cv.wait(lk);
        }
        if (!id) break;
        auto it = c->tickets.find(id);
        it->second.state = 1;
        if (c->budget) {
            c->used += fp;
            c->reserved += fp;
        }
        Ctx::Ticket t = it->second;
        lk.unlock();
        Reservation rv{c, fp};
        t_reservation = c->budget ? &rv : nullptr;
        t_serving = true;
        lrep_stats_t stats{};
        const int rc = solve(t.op, st, t.req.nev, t.req.block, t.req.tol, &t.req.opts, t.req.lambda, t.req.X,
                             t.req.Y, t.req.ldxy, &stats);
        t_serving = false;
        t_reservation = nullptr;
        lk.lock();
        if (c->budget) {
            c->used -= rv.left;   // the part of the reservation the solve did not take
            c->reserved -= fp;
        }
        auto it2 = c->tickets.find(id);
        if (it2 != c->tickets.end()) {
            it2->second.state = 2;
            it2->second.rc = rc;
            it2->second.stats = stats;
        }
        c->q_cv.notify_all();
    }
    lk.unlock();
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
}

}  // namespace

extern "C" {

int lrep_version(void) { return 100; }

const char* lrep_strerror(int code) {
    switch (code) {
        case LREP_OK: return "success";
        case LREP_EINVAL: return "invalid argument";
        case LREP_ENOMEM: return "out of device memory or HBM budget";
        case LREP_ENOTCONV: return "not converged within maxit";
        case LREP_EBREAKDOWN: return "biorthogonalisation breakdown";
        case LREP_ENOTSPD: return "operator not positive definite on the subspace";
        case LREP_ENUMERIC: return "non-finite value";
        case LREP_EDEVICE: return "HIP runtime error";
        case LREP_EAGAIN: return "request pending";
        case LREP_ECANCELED: return "request cancelled";
        default: return "unknown error";
    }
}

const char* lrep_last_error(lrep_ctx_t ctx) {
    if (!ctx) return "";
    std::lock_guard<std::mutex> g(ctx->err_mu);
    return ctx->last_error.c_str();
}

int lrep_init(lrep_ctx_t* out, int device, size_t hbm_budget_bytes, void* hip_stream) {
    if (!out) return LREP_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return LREP_EINVAL;
    auto* c = new lrep_ctx_s();
    c->device = device;
    c->budget = hbm_budget_bytes;
    if (set_device(c) != LREP_OK || noalloc_setup(device) != LREP_OK) {
        delete c;
        return LREP_EDEVICE;
    }
    if (hip_stream) {
        c->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return LREP_EDEVICE;
        }
        c->own_stream = true;
    }
    *out = c;
    return LREP_OK;
}

int lrep_finalize(lrep_ctx_t c) {
    if (!c) return LREP_EINVAL;
    {
        std::lock_guard<std::mutex> g(c->q_mu);
        c->stopping = true;
        for (auto& kv : c->tickets)
            if (kv.second.state == 0) kv.second.state = 3;
        c->queue.clear();
    }
    c->q_cv.notify_all();
    for (auto& t : c->workers) t.join();
    (void)hipSetDevice(c->device);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return LREP_OK;
}

int lrep_create_dense(lrep_ctx_t c, int64_t n, const double* K, const double* M, int64_t ld, uint32_t flags,
                      lrep_op_t* out) {
    if (!c || !out || !K || !M || n < 1 || ld < n || n > (int64_t)INT32_MAX) return LREP_EINVAL;
    *out = nullptr;
    if (set_device(c) != LREP_OK) return LREP_EDEVICE;
    auto* op = new lrep_op_s();
    op->ctx = c;
    op->n = n;
    op->kind = 0;
    op->flags = flags;
    const bool dev = flags & LREP_DEVICE_PTR;
    const bool borrow = dev && (flags & LREP_BORROW) && !(flags & LREP_INPUT_AB);
    if (borrow) {
        op->K = const_cast<double*>(K);
        op->M = const_cast<double*>(M);
        op->ld = ld;
    } else {
        const size_t bytes = (size_t)n * n * sizeof(double);
        int rc = op->Kbuf.alloc(c, bytes);
        if (rc == LREP_OK) rc = op->Mbuf.alloc(c, bytes);
        if (rc != LREP_OK) {
            delete op;
            return rc;
        }
        op->K = op->Kbuf.p;
        op->M = op->Mbuf.p;
        op->ld = n;
        const hipMemcpyKind kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
        hipError_t e = hipMemcpy2DAsync(op->K, n * sizeof(double), K, ld * sizeof(double), n * sizeof(double), n,
                                        kind, c->stream);
        if (e == hipSuccess)
            e = hipMemcpy2DAsync(op->M, n * sizeof(double), M, ld * sizeof(double), n * sizeof(double), n, kind,
                                 c->stream);
        if (e == hipSuccess && (flags & LREP_INPUT_AB)) e = combine_ab(c->stream, n, op->K, op->M);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) {
            c->set_error(hipGetErrorString(e));
            delete op;
            return LREP_EDEVICE;
        }
    }
    *out = op;
    return LREP_OK;
}

int lrep_create_callback(lrep_ctx_t c, int64_t n, lrep_apply_fn apply, void* user, uint32_t flags,
                         lrep_op_t* out) {
    if (!c || !out || !apply || n < 1 || n > (int64_t)INT32_MAX) return LREP_EINVAL;
    *out = nullptr;
    auto* op = new lrep_op_s();
    op->ctx = c;
    op->n = n;
    op->kind = 2;
    op->flags = flags;
    op->apply_fn = apply;
    op->apply_user = user;
    *out = op;
    return LREP_OK;
}

int lrep_create_lowrank(lrep_ctx_t c, int64_t n, int64_t rank, const double* delta, const double* L, int64_t ldl,
                        uint32_t flags, lrep_op_t* out) {
    if (!c || !out || !delta || n < 1 || rank < 0 || (rank > 0 && (!L || ldl < n)) || n > (int64_t)INT32_MAX)
        return LREP_EINVAL;
    *out = nullptr;
    if (set_device(c) != LREP_OK) return LREP_EDEVICE;
    auto* op = new lrep_op_s();
    op->ctx = c;
    op->n = n;
    op->kind = 1;
    op->flags = flags;
    op->rank = rank;
    const bool dev = flags & LREP_DEVICE_PTR;
    if (dev && (flags & LREP_BORROW)) {
        op->delta = const_cast<double*>(delta);
        op->L = const_cast<double*>(L);
        op->ldl = ldl;
    } else {
        int rc = op->dbuf.alloc(c, n * sizeof(double));
        if (rc == LREP_OK && rank > 0) rc = op->Lbuf.alloc(c, (size_t)n * rank * sizeof(double));
        if (rc != LREP_OK) {
            delete op;
            return rc;
        }
        op->delta = op->dbuf.p;
        op->L = op->Lbuf.p;
        op->ldl = n;
        const hipMemcpyKind kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
        hipError_t e = hipMemcpyAsync(op->delta, delta, n * sizeof(double), kind, c->stream);
        if (e == hipSuccess && rank > 0)
            e = hipMemcpy2DAsync(op->L, n * sizeof(double), L, ldl * sizeof(double), n * sizeof(double), rank, kind,
                                 c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) {
            c->set_error(hipGetErrorString(e));
            delete op;
            return LREP_EDEVICE;
        }
    }
    // row-major copy of L for the streaming M apply (when the HBM budget
    // allows it; without it the column-major passes are used)
    if (rank >= 1 && rank <= 256 &&
        op->Lrbuf.alloc(c, (size_t)n * lowrank_row_ld(rank) * sizeof(double)) == LREP_OK) {
        hipError_t e = lowrank_make_rows(c->stream, (int)n, (int)rank, op->L, op->ldl, op->Lrbuf.p);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) {
            c->set_error(hipGetErrorString(e));
            delete op;
            return LREP_EDEVICE;
        }
        op->Lr = op->Lrbuf.p;
    }
    *out = op;
    return LREP_OK;
}

int lrep_set_nullspace(lrep_op_t op, int64_t r, const double* X0, int64_t ld, int32_t on_device) {
    if (!op || r < 0 || r >= op->n || (r > 0 && (!X0 || ld < op->n))) return LREP_EINVAL;
    Ctx* c = op->ctx;
    if (set_device(c) != LREP_OK) return LREP_EDEVICE;
    op->r0 = 0;
    op->X0.release();
    op->Y0.release();
    if (r == 0) return LREP_OK;
    DevBuf tmp;
    int rc = tmp.alloc(c, (size_t)op->n * r * sizeof(double));
    if (rc != LREP_OK) return rc;
    hipError_t e = hipMemcpy2DAsync(tmp.p, op->n * sizeof(double), X0, ld * sizeof(double), op->n * sizeof(double), r,
                                    on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return LREP_EDEVICE;
    // with a metric B = C C^T the scaled operator's null space is C^T N(K)
    if (op->has_metric()) {
        DevBuf t2, wk;
        const size_t welems = op->MetLT.p ? (size_t(8) << 20) : 0;
        if (op->MetLT.p) {
            rc = t2.alloc(c, (size_t)op->n * r * sizeof(double));
            if (rc == LREP_OK) rc = wk.alloc(c, welems * sizeof(double));
            if (rc != LREP_OK) return rc;
        }
        rc = op_metric_transform(op, c->stream, true, (int)r, tmp.p, op->n, t2.p, wk.p, welems);
        if (rc != LREP_OK) return rc;
    }
    rc = prepare_nullspace(op, c->stream, r, tmp.p);
    if (rc != LREP_OK) {
        op->r0 = 0;
        op->X0.release();
        op->Y0.release();
    }
    return rc;
}

int lrep_xy_to_uv(lrep_ctx_t c, int64_t n, int64_t nev, const double* X, const double* Y, int64_t ldxy, double* U,
                  double* V, int64_t lduv) {
    if (!c || n < 1 || nev < 0 || n > (int64_t)INT32_MAX || nev > 65535 || ldxy < n || lduv < n || !X || !Y || !U ||
        !V)
        return LREP_EINVAL;
    if (set_device(c) != LREP_OK) return LREP_EDEVICE;
    hipError_t e = xy_to_uv(c->stream, (int)n, (int)nev, X, Y, ldxy, U, V, lduv);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        c->set_error(hipGetErrorString(e));
        return LREP_EDEVICE;
    }
    return LREP_OK;
}

int lrep_find_nullspace(lrep_op_t op, int64_t rmax, double tol, uint64_t seed, int64_t* r_out, double* res_out) {
    if (!op || !r_out || rmax < 1 || rmax > 64 || rmax >= op->n || !(tol > 0)) return LREP_EINVAL;
    Ctx* c = op->ctx;
    if (set_device(c) != LREP_OK) return LREP_EDEVICE;
    double res = 0.0;
    *r_out = 0;
    const int rc = find_nullspace(op, c->stream, rmax, tol, seed, r_out, &res);
    if (res_out) *res_out = res;
    return rc;
}

int lrep_set_metric(lrep_op_t op, int64_t n_b, const double* b, uint32_t flags) {
    if (!op || !b || n_b != op->n) return LREP_EINVAL;
    Ctx* c = op->ctx;
    if (set_device(c) != LREP_OK) return LREP_EDEVICE;
    auto refuse = [&](const char* why) {
        c->set_error(why);
        return LREP_EINVAL;
    };
    if (op->kind == 2) return refuse("lrep_set_metric: a callback operator applies the scaled pencil itself");
    if (op->has_metric()) return refuse("lrep_set_metric: the operator already has a metric");
    if (op->r0 > 0) return refuse("lrep_set_metric: set the metric before the null space");
    const bool owned = op->kind == 0 ? (op->K == op->Kbuf.p && op->M == op->Mbuf.p)
                                     : (op->delta == op->dbuf.p && (op->rank == 0 || op->L == op->Lbuf.p));
    if (!owned) return refuse("lrep_set_metric: the operator borrows the caller's arrays");
    const int64_t n = op->n;
    DevBuf sb, bb, flag;
    int rc = sb.alloc(c, (size_t)n * sizeof(double));
    if (rc == LREP_OK && !(flags & LREP_DEVICE_PTR)) rc = bb.alloc(c, (size_t)n * sizeof(double));
    if (rc == LREP_OK) rc = flag.alloc(c, sizeof(double));
    if (rc != LREP_OK) return rc;
    const double* bd = b;
    int* bad = reinterpret_cast<int*>(flag.p);
    hipError_t e = hipSuccess;
    if (!(flags & LREP_DEVICE_PTR)) {
        e = hipMemcpyAsync(bb.p, b, (size_t)n * sizeof(double), hipMemcpyHostToDevice, c->stream);
        bd = bb.p;
    }
    if (e == hipSuccess) e = hipMemsetAsync(bad, 0, sizeof(int), c->stream);
    if (e == hipSuccess) e = metric_prepare(c->stream, n, bd, sb.p, bad);
    int hbad = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        c->set_error(hipGetErrorString(e));
        return LREP_EDEVICE;
    }
    if (hbad) return refuse("lrep_set_metric: every entry of b must be positive and finite");
    const double* sv = sb.p;
    if (op->kind == 0) {
        e = metric_scale_sym(c->stream, n, op->K, op->ld, sv);
        if (e == hipSuccess) e = metric_scale_sym(c->stream, n, op->M, op->ld, sv);
        // 16-bit copies, if any, were made from the unscaled operator
        std::lock_guard<std::mutex> lk(op->mu16);
        op->prec16 = 0;
        op->K16buf.release();
        op->M16buf.release();
    } else {
        e = metric_scale_diag(c->stream, n, op->delta, sv);
        if (e == hipSuccess && op->rank > 0) e = metric_scale_rows(c->stream, n, (int)op->rank, op->L, op->ldl, sv, false);
        if (e == hipSuccess && op->Lr) e = lowrank_make_rows(c->stream, (int)n, (int)op->rank, op->L, op->ldl, op->Lr);
        // an FP32 copy, if any, was made from the unscaled rows
        std::lock_guard<std::mutex> lk(op->mu16);
        op->Lr32buf.release();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        c->set_error(hipGetErrorString(e));
        return LREP_EDEVICE;
    }
    op->Sbuf.take(sb);
    op->Sv = op->Sbuf.p;
    return LREP_OK;
}

int lrep_set_metric_dense(lrep_op_t op, int64_t n_b, const double* B, int64_t ldb, uint32_t flags) {
    if (!op || !B || n_b != op->n || ldb < op->n) return LREP_EINVAL;
    Ctx* c = op->ctx;
    if (set_device(c) != LREP_OK) return LREP_EDEVICE;
    auto refuse = [&](const char* why) {
        c->set_error(why);
        return LREP_EINVAL;
    };
    if (op->kind != 0) return refuse("lrep_set_metric_dense: only dense operators keep their structure under a dense metric");
    if (op->has_metric()) return refuse("lrep_set_metric_dense: the operator already has a metric");
    if (op->r0 > 0) return refuse("lrep_set_metric_dense: set the metric before the null space");
    if (!(op->K == op->Kbuf.p && op->M == op->Mbuf.p))
        return refuse("lrep_set_metric_dense: the operator borrows the caller's arrays");
    const int64_t n = op->n;
    const size_t sq = (size_t)n * n * sizeof(double);
    const size_t welems = size_t(8) << 20;
    DevBuf Lb, Xb, LT, LinvT, Tb, Vall, Wb, Pt, wk, flag;
    int rc = Lb.alloc(c, sq);
    if (rc == LREP_OK) rc = Xb.alloc(c, sq);
    if (rc == LREP_OK) rc = LT.alloc(c, sq);
    if (rc == LREP_OK) rc = LinvT.alloc(c, sq);
    if (rc == LREP_OK) rc = Tb.alloc(c, (size_t)n * 64 * sizeof(double));
    if (rc == LREP_OK) rc = Vall.alloc(c, (size_t)n * 64 * sizeof(double) + 64 * 64 * sizeof(double));
    if (rc == LREP_OK) rc = Wb.alloc(c, 64 * 64 * sizeof(double));
    if (rc == LREP_OK) rc = Pt.alloc(c, (size_t)n * 64 * sizeof(double));
    if (rc == LREP_OK) rc = wk.alloc(c, welems * sizeof(double));
    if (rc == LREP_OK) rc = flag.alloc(c, sizeof(double));
    if (rc != LREP_OK) return rc;
    int* bad = reinterpret_cast<int*>(flag.p);
    hipError_t e = hipMemcpy2DAsync(Lb.p, n * sizeof(double), B, ldb * sizeof(double), n * sizeof(double), n,
                                    (flags & LREP_DEVICE_PTR) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                                    c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(bad, 0, sizeof(int), c->stream);
    if (e == hipSuccess)
        e = metric_dense_setup(c->stream, n, Lb.p, Xb.p, Tb.p, LT.p, LinvT.p, Vall.p, Wb.p, Pt.p, wk.p, welems, bad);
    int hbad = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        c->set_error(hipGetErrorString(e));
        return LREP_EDEVICE;
    }
    if (hbad) return refuse("lrep_set_metric_dense: B is not positive definite (Cholesky pivot <= 0)");
    // K <- L^-1 K L^-T, M <- L^-1 M L^-T (Lb is free now: L^T is kept in LT)
    e = metric_dense_apply(c->stream, n, op->K, op->ld, Xb.p, LinvT.p, Lb.p, wk.p, welems);
    if (e == hipSuccess) e = metric_dense_apply(c->stream, n, op->M, op->ld, Xb.p, LinvT.p, Lb.p, wk.p, welems);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    {
        std::lock_guard<std::mutex> lk(op->mu16);
        op->prec16 = 0;
        op->K16buf.release();
        op->M16buf.release();
    }
    if (e != hipSuccess) {
        // K and M may be partly transformed: the operator is no longer usable
        c->set_error(std::string("lrep_set_metric_dense: ") + hipGetErrorString(e));
        return LREP_EDEVICE;
    }
    op->MetLT.take(LT);
    op->MetLinvT.take(LinvT);
    return LREP_OK;
}

int lrep_destroy_op(lrep_op_t op) {
    if (!op) return LREP_EINVAL;
    (void)set_device(op->ctx);
    (void)hipStreamSynchronize(op->ctx->stream);
    delete op;
    return LREP_OK;
}

int lrep_solve(lrep_op_t op, int64_t n, int64_t nev, int64_t block, double tol, const lrep_solve_opts_t* opts,
               double* lambda, double* X, double* Y, int64_t ldxy, lrep_stats_t* stats) {
    if (!op) return LREP_EINVAL;
    if (n != op->n) return LREP_EINVAL;
    if (set_device(op->ctx) != LREP_OK) return LREP_EDEVICE;
    return solve(op, op->ctx->stream, nev, block, tol, opts, lambda, X, Y, ldxy, stats);
}

int lrep_submit(lrep_ctx_t c, lrep_op_t op, const lrep_request_t* req, lrep_ticket_t* ticket) {
    if (!c || !op || !req || !ticket || op->ctx != c) return LREP_EINVAL;
    if (req->nev < 1 || req->block < 1 || !(req->tol > 0) || !req->lambda || !req->X || !req->Y ||
        req->ldxy < op->n)
        return LREP_EINVAL;
    size_t fp = 0;
    const int frc = solve_footprint(op, req->nev, req->block, req->tol, &req->opts, &fp, true);
    if (frc != LREP_OK) return frc;
    std::lock_guard<std::mutex> g(c->q_mu);
    if (c->stopping) return LREP_EINVAL;
    if (c->broken) return LREP_EDEVICE;
    if (c->workers.empty()) {
        c->n_workers = 4;
        for (int i = 0; i < c->n_workers; ++i) c->workers.emplace_back(worker_main, c);
    }
    const uint64_t id = c->next_ticket++;
    Ctx::Ticket t{};
    t.op = op;
    t.req = *req;
    t.state = 0;
    t.rc = LREP_EAGAIN;
    t.footprint = fp;
    c->tickets[id] = t;
    c->queue.push_back(id);
    *ticket = id;
    c->q_cv.notify_all();
    return LREP_OK;
}

int lrep_poll(lrep_ctx_t c, lrep_ticket_t ticket, lrep_stats_t* stats_out) {
    if (!c) return LREP_EINVAL;
    std::lock_guard<std::mutex> g(c->q_mu);
    auto it = c->tickets.find(ticket);
    if (it == c->tickets.end()) return LREP_EINVAL;
    if (it->second.state == 0 || it->second.state == 1) return LREP_EAGAIN;
    const int rc = it->second.state == 3 ? LREP_ECANCELED : it->second.rc;
    if (stats_out) *stats_out = it->second.stats;
    c->tickets.erase(it);
    return rc;
}

int lrep_cancel(lrep_ctx_t c, lrep_ticket_t ticket) {
    if (!c) return LREP_EINVAL;
    std::lock_guard<std::mutex> g(c->q_mu);
    auto it = c->tickets.find(ticket);
    if (it == c->tickets.end()) return LREP_EINVAL;
    if (it->second.state != 0) return LREP_EAGAIN;   // running or finished: not interrupted
    it->second.state = 3;
    c->queue.erase(std::remove(c->queue.begin(), c->queue.end(), ticket), c->queue.end());
    return LREP_OK;
}

}  // extern "C"
