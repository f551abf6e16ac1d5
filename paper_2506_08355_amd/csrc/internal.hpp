// Library-internal objects behind the C ABI (lrep.h).
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/lrep.h"
#include "kernels.hpp"

namespace lrep {

struct Ctx;
struct CgJob;   // a served Step-6 CG solve waiting to be batched (solver.hip)

// A served request's admission reserves its whole footprint against the
// context's budget before the solve starts; the solve's own allocations (on
// the worker thread) are then taken from that reservation.
struct Reservation {
    Ctx* ctx;
    size_t left;
};
extern thread_local Reservation* t_reservation;
// true on a serving worker thread while it runs a request's solve
extern thread_local bool t_serving;

// Device allocation charged against the context's HBM budget.
struct DevBuf {
    Ctx* ctx = nullptr;
    double* p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf();
    int alloc(Ctx* c, size_t nbytes);   // LREP_OK / LREP_ENOMEM / LREP_EDEVICE
    void release();
    // take over o's allocation (o is left empty)
    void take(DevBuf& o) {
        release();
        ctx = o.ctx;
        p = o.p;
        bytes = o.bytes;
        o.ctx = nullptr;
        o.p = nullptr;
        o.bytes = 0;
    }
};

struct Op {
    Ctx* ctx = nullptr;
    int64_t n = 0;
    int kind = 0;              // 0 dense, 1 low rank, 2 caller-supplied products
    uint32_t flags = 0;
    // dense
    double* K = nullptr;
    double* M = nullptr;
    int64_t ld = 0;
    DevBuf Kbuf, Mbuf;
    // low rank: K = diag(delta), M = diag(delta) + 2 L L^T
    double* delta = nullptr;
    double* L = nullptr;
    int64_t rank = 0, ldl = 0;
    DevBuf dbuf, Lbuf;
    // row-major copy of L (n x lowrank_row_ld(rank)) for the streaming M apply
    DevBuf Lrbuf;
    double* Lr = nullptr;
    // caller-supplied products
    lrep_apply_fn apply_fn = nullptr;
    void* apply_user = nullptr;
    // diagonal metric B = diag(b) of a generalized LREP: Sv = b^-1/2 (device,
    // n values); the operator data above is already the scaled S K S, S M S
    DevBuf Sbuf;
    double* Sv = nullptr;
    // dense SPD metric B = L L^T (dense operators): L^T and L^-T (n x n, ld n);
    // the operator data is already L^-1 K L^-T, L^-1 M L^-T
    DevBuf MetLT, MetLinvT;
    bool has_metric() const { return Sv != nullptr || MetLT.p != nullptr; }
    // generalized null space, biorthonormal X0^T Y0 = I (roles already exchanged)
    int64_t r0 = 0;
    DevBuf X0, Y0;
    // 16-bit copies of a dense K and M for the mixed-precision CG applies
    // (precision 1: BF16, 2: FP16), made on first use
    std::mutex mu16;
    int prec16 = 0;
    DevBuf K16buf, M16buf;
    // FP32 copy of the rows of L for the fused CG passes (precision 4), made on
    // first use (under mu16); dropped when the operator data changes
    DevBuf Lr32buf;
    const float* Lr32() const { return reinterpret_cast<const float*>(Lr32buf.p); }
    const uint16_t* K16() const { return reinterpret_cast<const uint16_t*>(K16buf.p); }
    const uint16_t* M16() const { return reinterpret_cast<const uint16_t*>(M16buf.p); }
    bool null_on_M() const { return (flags & LREP_NULL_ON_M) != 0; }
    // serving: Step-6 CG solves of concurrent requests waiting to run as one
    // block CG (solver.hip, Solver::cg_batched)
    std::mutex batch_mu;
    std::condition_variable batch_cv;
    std::vector<CgJob*> batch_queue;
    bool batch_running = false;
};

struct Ctx {
    int device = 0;
    size_t budget = 0;         // 0: unlimited
    std::atomic<size_t> used{0};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::mutex err_mu;
    std::string last_error;
    // serving
    struct Ticket {
        lrep_op_t op;
        lrep_request_t req;
        int state;             // 0 queued, 1 running, 2 done, 3 cancelled
        int rc;
        lrep_stats_t stats;
        size_t footprint;      // device bytes the solve charges (admission)
    };
    // bytes reserved for the requests now running (each its whole footprint
    // from admission to completion); used - reserved is what the operators
    // and other allocations hold
    size_t reserved = 0;
    bool broken = false;       // a worker could not start: submit fails
    std::mutex q_mu;
    std::condition_variable q_cv;
    std::map<uint64_t, Ticket> tickets;
    std::deque<uint64_t> queue;
    uint64_t next_ticket = 1;
    std::vector<std::thread> workers;
    bool stopping = false;
    int n_workers = 0;
    void set_error(const std::string& s) {
        std::lock_guard<std::mutex> g(err_mu);
        last_error = s;
    }
};

// Solver entry (solver.hip).  `st` is the stream the solve runs on.
int solve(Op* op, hipStream_t st, int64_t nev, int64_t block, double tol, const lrep_solve_opts_t* opts,
          double* lambda, double* X, double* Y, int64_t ldxy, lrep_stats_t* stats);

// Device bytes a solve with these arguments charges to the context (its
// workspaces, and 16-bit operator copies it would make); LREP_EINVAL for
// arguments the solve would reject.  No device work.
int solve_footprint(Op* op, int64_t nev, int64_t block, double tol, const lrep_solve_opts_t* opts, size_t* bytes,
                    bool served = false);

// Null-space preparation (solver.hip): X0t (device, n x r, ld n) -> op->X0, op->Y0.
int prepare_nullspace(Op* op, hipStream_t st, int64_t r, const double* X0t_dev);
// Coordinate change of n x cols blocks for an operator with a metric B = C C^T:
// to_hat x^ = C^T x, else x = C^-T x^ (in place; tmp n x cols, ld n, used by a
// dense metric).  No-op without a metric.
int op_metric_transform(Op* op, hipStream_t st, bool to_hat, int cols, double* X, int64_t ldx, double* tmp,
                        double* work, size_t work_elems);

// A basis of the null space of the semidefinite operator (at most rmax
// columns), then prepare_nullspace on it; *r_out its dimension, *res_out the
// largest ||A z|| / ||A||_est of the orthonormal basis vectors.
int find_nullspace(Op* op, hipStream_t st, int64_t rmax, double tol, uint64_t seed, int64_t* r_out,
                   double* res_out);

// Operator apply with the roles (after a possible exchange): which = 0 -> "K", 1 -> "M".
// With pq (low-rank operators, cols <= 32, op_apply_has_pq true), also
// pq[t * 32 + j] = the sum over the 64-row tile t of X[:, j] Y[:, j].
int op_apply(Op* op, hipStream_t st, int which, const double* X, int64_t ldx, int cols, double* Y, int64_t ldy,
             double* work, size_t work_elems, double* small, const int* active_flag,
             hipEvent_t* ev = nullptr, double* pq = nullptr);
bool op_apply_has_pq(const Op* op, int which, const double* X, int64_t ldx, int cols);
// device address of the allocation-free apply's fixed scratch array, looked
// up once per device (noalloc.hip); called by lrep_init with the device current
int noalloc_setup(int device);

}  // namespace lrep
