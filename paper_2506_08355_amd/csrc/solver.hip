// BOSP driver on one HIP stream (Algorithm "BOSP algorithm", Sections 3.2-3.3).
//
// Device data layout (column-major FP64; the basis, locked and Step-6 blocks
// use the padded leading dimension ldn = solver_ld(n), whose byte stride is
// not a multiple of 2 KiB, so that the columns of a block do not all start on
// the same HBM channel; the CG state uses n):
//   buf[2] x {X, Y, KX, MY}   n x cap, cap = b + 4w + 1 columns.  The current
//                             subspace U = [X~, P~, W~] (and V, K U, M V) sits
//                             in one buffer at a column offset; the Ritz
//                             pull-back of each iteration is written into the
//                             other buffer, where P~ and W~ are appended so
//                             that the next subspace needs no copy.
//   Xc, Yc                    n x nev locked (converged) pairs.
//   X0, Y0                    n x r generalized null space (on the operator).
//   CG state                  n x w each (solution, residual, direction, A p).
// Small matrices (d <= 128) stay on the device; per iteration the host reads
// back only the Ritz values, the Step-4 residuals and a few status words.
//
// What differs from the paper's own (CPU) design, and why:
//   * MGS-Biorth of a block runs as two passes of "Gram matrix, then the
//     MGS-Biorth recurrence on coefficient vectors, then one block product"
//     (block form sanctioned by the paper's remark on level-3 BLAS); the
//     column-by-column form needs w(w-1) grid-wide reductions per block.
//   * the small problem's SVD is a one-sided Jacobi iteration in one
//     workgroup (the paper uses a LAPACK SVD on the CPU).
//   * K U and M V are applied afresh to the whole subspace only every
//     `refresh` iterations (the paper's cost model re-applies them every
//     iteration, 2d mat-vecs per Step 3); in between they follow the basis
//     through the same coefficient products, and only the new W~, Z~ block
//     is applied.  They are fresh again after every restoration of
//     biorthogonality and before any pair is locked or returned.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "internal.hpp"

#define CK(x)                                  \
    do {                                       \
        hipError_t e_ = (x);                   \
        if (e_ != hipSuccess) return dev_fail(e_, #x); \
    } while (0)
#define CR(x)                     \
    do {                          \
        int r_ = (x);             \
        if (r_ != LREP_OK) return r_; \
    } while (0)

namespace lrep {

// A Step-6 CG solve waiting to run in a block CG shared with other served
// requests on the same operator (Solver::cg_batched).
struct CgJob {
    const void* owner;      // the Solver whose job it is
    int which, nw, maxit, precision, fused;
    double tol;
    const double* B;        // right-hand sides (device, ld ldb)
    int64_t ldb;
    double* X;              // the owner's CG solution block (device, n x nw, ld n)
    hipEvent_t ready;       // recorded on the owner's stream once B is written
    hipEvent_t done;        // recorded on the running stream once X is written
    int rc = LREP_OK;
    bool finished = false;
    bool shared = false;    // ran together with other requests' columns
    bool compatible(const CgJob& o) const {
        return which == o.which && maxit == o.maxit && tol == o.tol && precision == o.precision && fused == o.fused;
    }
};

namespace {

constexpr double MGS_COS_TOL = 1e-10;
constexpr double MGS_DEP_TOL = 1e-13;
// In coefficient space a column norm comes from a Gram matrix, which resolves
// ||p~|| / ||x|| only down to about sqrt(eps); the dependence test there uses
// this floor instead of MGS_DEP_TOL.
constexpr double MGS_DEP_TOL_COEF = 1e-7;
constexpr size_t GEMM_WORK_ELEMS = size_t(8) << 20;   // 64 MiB of split partials

struct HostStatus {
    double eps[kMaxD];
    double lam[kMaxD];
    double offmax;
    double drift;
    int status[ST_COUNT];
    unsigned long long napplies[2];
};

// leading dimension of the solver's n-row blocks: n rounded up to 32 doubles,
// plus 32 more when that is a multiple of 256 (a power-of-two stride puts the
// same row of every column on the same memory channel; measured 30% on the
// Gram products at n = 2^18)
int64_t solver_ld(int64_t n) {
    int64_t ld = (n + 31) / 32 * 32;
    if (ld % 256 == 0) ld += 32;
    return ld;
}

struct Solver {
    Op* op;
    hipStream_t st;
    int64_t n;
    // served Step-6 CG solves may run batched with other requests' (set by
    // solve_configure; the CG buffers then hold 32 columns)
    bool batch = false;
    DevBuf bcomb;                                  // gathered right-hand sides of a batch (n x 32, ld n)
    hipEvent_t ev_ready = nullptr, ev_done = nullptr;
    int64_t ldn = 0;   // leading dimension of the blocks (solver_ld(n), set by buffers())
    int b, w, cap, nev, r0;
    double tol;
    lrep_solve_opts_t o{};
    // device buffers
    DevBuf bX[2], bY[2], bKX[2], bMY[2];
    DevBuf Xc, Yc;
    DevBuf cgX, cgR, cgP, cgQ, Zs, Ws, rhs, tX, tY;
    DevBuf gwork, dsmall, ismall;
    // carved small buffers
    double *Kh, *Mh, *S, *Xh, *Yh, *lam, *eps, *lamw, *Ph, *Qh, *Acoef, *Bcoef, *scr, *G, *Cproj, *Tlr, *part,
        *cg_rr, *cg_bb, *cg_alpha, *cg_beta, *offmax, *cg_pq, *cg_c, *cg_T;
    int64_t kproj;
    int *status, *win, *wincol, *cg_active, *cg_any;
    unsigned* tickets;
    unsigned long long* napplies;
    HostStatus* hs = nullptr;
    // host-visible CG note (mapped, coherent pinned memory) and its device alias
    unsigned long long* note_h = nullptr;
    unsigned long long* note_d = nullptr;
    unsigned long long cg_seq = 0;
    std::string err;
    lrep_stats_t stats{};
    // profiling of the CG applies: event pairs, column counts and the CG
    // "any column active" flag logged on the device just before each apply
    std::vector<hipEvent_t> prof_ev;
    std::vector<int> prof_cols;
    std::vector<double> prof_b, prof_f;   // algorithmic bytes and flops of each timed launch
    DevBuf prof_log;
    static constexpr int kProfMax = 1 << 16;

    // Step-6 graphs, one per (block width, basis buffer)
    struct Step6Graph {
        int nw;
        const double* nx;
        hipGraphExec_t exec;
    };
    std::vector<Step6Graph> graphs6;
    bool capturing = false;
    hipEvent_t np_ev = nullptr;   // Step 5's status copy has landed

    ~Solver() {
        for (auto& g : graphs6) (void)hipGraphExecDestroy(g.exec);
        if (np_ev) (void)hipEventDestroy(np_ev);
        if (ev_ready) (void)hipEventDestroy(ev_ready);
        if (ev_done) (void)hipEventDestroy(ev_done);
        if (hs) (void)hipHostFree(hs);
        if (note_h) (void)hipHostFree(note_h);
        for (auto e : prof_ev) (void)hipEventDestroy(e);
        for (auto e : mark_pool) (void)hipEventDestroy(e);
    }

    // events for the next timed apply; the "any column active" flag is
    // logged by the caller's kernel into *slot when slot != nullptr, else
    // copied here
    hipEvent_t* prof_next(int cols, int** slot = nullptr, int prec = 0, bool fused = false) {
        const size_t i = prof_cols.size();
        if (!prof_log.p || i >= (size_t)kProfMax) return nullptr;
        while (prof_ev.size() < 2 * (i + 1)) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            prof_ev.push_back(e);
        }
        int* log = reinterpret_cast<int*>(prof_log.p);
        if (slot) {
            *slot = log + i;
        } else if (hipMemcpyAsync(log + i, cg_any, sizeof(int), hipMemcpyDeviceToDevice, st) != hipSuccess) {
            return nullptr;
        }
        prof_cols.push_back(cols);
        const double nn = (double)n, c = cols;
        if (op->kind == 0 && prec != 0) {   // 16-bit operator and block (3 parts each for BF16x3), FP64 result
            const double parts = prec == 3 ? 3.0 : 1.0;
            prof_b.push_back(parts * (2.0 * nn * nn + 2.0 * nn * c) + 8.0 * nn * c);
            prof_f.push_back(2.0 * nn * nn * c);
        } else if (op->kind == 0) {
            prof_b.push_back(8.0 * nn * nn + 16.0 * nn * c);
            prof_f.push_back(2.0 * nn * nn * c);
        } else if (op->kind == 2) {   // caller-supplied products: no byte model
            prof_b.push_back(0.0);
            prof_f.push_back(0.0);
        } else if (fused) {   // fused low-rank M step: L once (FP64 or FP32 rows); x, r, p read and written; delta
            const double r = (double)op->rank;
            prof_b.push_back((o.precision == 4 ? 4.0 : 8.0) * nn * r + 48.0 * nn * c + 8.0 * nn);
            prof_f.push_back(4.0 * nn * r * c + 14.0 * nn * c);
        } else {   // low-rank M: L read twice, Y read twice, result written once
            const double r = (double)op->rank;
            prof_b.push_back(16.0 * nn * r + 24.0 * nn * c);
            prof_f.push_back(4.0 * nn * r * c + 3.0 * nn * c);
        }
        return &prof_ev[2 * i];
    }

    int prof_collect() {
        const size_t k = prof_cols.size();
        if (k == 0) return LREP_OK;
        std::vector<int> log(k);
        CK(hipMemcpyAsync(log.data(), prof_log.p, k * sizeof(int), hipMemcpyDeviceToHost, st));
        CK(hipStreamSynchronize(st));
        const double nn = (double)n;
        for (size_t i = 0; i < k; ++i) {
            if (!log[i]) continue;   // every column had converged: the launch returned at once
            float ms = 0.f;
            CK(hipEventElapsedTime(&ms, prof_ev[2 * i], prof_ev[2 * i + 1]));
            stats.prof_launches++;
            stats.prof_ms += ms;
            stats.prof_bytes += prof_b[i];
            stats.prof_flops += prof_f[i];
        }
        return LREP_OK;
    }

    // per-phase GPU time (opts.profile): an event marks where each phase
    // starts on the stream; the time to the next mark belongs to it
    std::vector<std::pair<int, hipEvent_t>> marks;
    std::vector<hipEvent_t> mark_pool;
    void mark(int phase) {
        if (!o.profile) return;
        hipEvent_t e;
        if (marks.size() < mark_pool.size()) {
            e = mark_pool[marks.size()];
        } else {
            if (hipEventCreate(&e) != hipSuccess) return;
            mark_pool.push_back(e);
        }
        if (hipEventRecord(e, st) == hipSuccess) marks.emplace_back(phase, e);
    }
    int collect_phases() {
        if (marks.size() < 2) return LREP_OK;
        CK(hipEventSynchronize(marks.back().second));
        for (size_t i = 0; i + 1 < marks.size(); ++i) {
            float ms = 0.f;
            CK(hipEventElapsedTime(&ms, marks[i].second, marks[i + 1].second));
            if (marks[i].first >= 0 && marks[i].first < 5) stats.phase_ms[marks[i].first] += ms;
        }
        return LREP_OK;
    }

    int fail(int code, const char* what) {
        err = what;
        return code;
    }
    int dev_fail(hipError_t e, const char* what) {
        err = std::string(what) + ": " + hipGetErrorString(e);
        return LREP_EDEVICE;
    }


    // layout of the small carved device arrays (offsets in doubles) and its size
    struct SmallLayout {
        size_t Kh, Mh, S, Xh, Yh, lam, eps, lamw, Ph, Qh, A, B, scr, G, C, T, part, rr, bb, al, be, om, pq, cc, cT;
        size_t total;
    };
    SmallLayout small_layout() const {
        const size_t D2 = (size_t)kMaxD * kMaxD;
        const int cw = std::max(w, 1);
        const int64_t kp = r0 + nev + cap + 8;
        const int64_t rank = op->kind == 1 ? op->rank : 0;
        size_t nd = 0;
        auto carve = [&](size_t cnt) {
            size_t o2 = nd;
            nd += (cnt + 31) & ~size_t(31);
            return o2;
        };
        SmallLayout l;
        l.Kh = carve(D2); l.Mh = carve(D2); l.S = carve(D2); l.Xh = carve(D2); l.Yh = carve(D2);
        l.lam = carve(kMaxD); l.eps = carve(kMaxD); l.lamw = carve(kMaxD); l.Ph = carve(kMaxD * 64);
        l.Qh = carve(kMaxD * 64); l.A = carve(D2); l.B = carve(2 * D2); l.scr = carve(4 * D2);
        l.G = carve(4 * D2); l.C = carve((size_t)kp * std::max(kMaxD, cw));
        l.T = carve((size_t)std::max<int64_t>(rank, 1) * kMaxD); l.part = carve((size_t)256 * kMaxD * 4);
        l.rr = carve(kMaxD); l.bb = carve(kMaxD); l.al = carve(kMaxD); l.be = carve(kMaxD); l.om = carve(8);
        l.pq = carve(cg_pq_elems((int)stream_tiles((int)n))); l.cc = carve(kMaxD);
        l.cT = carve(op->kind == 1 ? (size_t)256 * 32 : 32);
        l.total = nd;
        return l;
    }
    static size_t int_bytes() { return sizeof(int) * (8 + 3 * kMaxD + 8 + 8) + 4 * sizeof(unsigned long long); }

    // Every device buffer of a solve with its size, in allocation order; alloc()
    // allocates them, footprint() adds them up (the serving admission).
    template <class F>
    int buffers(F&& f) {
        // a caller-supplied product function gets contiguous blocks (ld n)
        ldn = op->kind == 2 ? n : solver_ld(n);
        const size_t col = (size_t)ldn * sizeof(double);
        for (int i = 0; i < 2; ++i) {
            CR(f(bX[i], col * cap));
            CR(f(bY[i], col * cap));
            CR(f(bKX[i], col * cap));
            CR(f(bMY[i], col * cap));
        }
        CR(f(Xc, col * nev));
        CR(f(Yc, col * nev));
        const size_t cw = (size_t)std::max(w, 1);
        // the CG state (ld n): 32 columns when the solve may lead a batch
        const size_t cwg = batch ? std::max<size_t>(cw, 32) : cw;
        const size_t coln = (size_t)n * sizeof(double);
        CR(f(cgX, std::max(col * cw, coln * cwg)));
        CR(f(cgR, std::max(col * cw, coln * cwg)));
        CR(f(cgP, std::max(col * cw, coln * cwg)));
        CR(f(cgQ, std::max(col * cw, coln * cwg)));
        if (batch) CR(f(bcomb, coln * 32));
        CR(f(Zs, col * cw));
        CR(f(Ws, col * cw));
        CR(f(rhs, col * cw));
        CR(f(tX, col * kMaxD));
        CR(f(tY, col * kMaxD));
        CR(f(gwork, GEMM_WORK_ELEMS * sizeof(double)));
        CR(f(dsmall, small_layout().total * sizeof(double)));
        CR(f(ismall, int_bytes()));
        if (o.profile) CR(f(prof_log, kProfMax * sizeof(int)));
        return LREP_OK;
    }

    // device bytes alloc() will charge to the context (DevBuf charges 8 for 0)
    size_t footprint() {
        size_t total = 0;
        (void)buffers([&](DevBuf&, size_t bytes) {
            total += bytes ? bytes : 8;
            return LREP_OK;
        });
        return total;
    }

    int alloc() {
        Ctx* c = op->ctx;
        CR(buffers([&](DevBuf& b, size_t bytes) { return b.alloc(c, bytes); }));
        kproj = r0 + nev + cap + 8;
        const SmallLayout l = small_layout();
        double* base = dsmall.p;
        Kh = base + l.Kh; Mh = base + l.Mh; S = base + l.S; Xh = base + l.Xh; Yh = base + l.Yh;
        lam = base + l.lam; eps = base + l.eps; lamw = base + l.lamw; Ph = base + l.Ph; Qh = base + l.Qh;
        Acoef = base + l.A; Bcoef = base + l.B; scr = base + l.scr; G = base + l.G; Cproj = base + l.C;
        Tlr = base + l.T; part = base + l.part; cg_rr = base + l.rr; cg_bb = base + l.bb; cg_alpha = base + l.al;
        cg_beta = base + l.be; offmax = base + l.om; cg_pq = base + l.pq; cg_c = base + l.cc; cg_T = base + l.cT;
        // ints: status(8) win(kMaxD) wincol(kMaxD) cg_active(kMaxD) cg_any(8) tickets(8) napplies(2 x u64)
        int* ib = reinterpret_cast<int*>(ismall.p);
        status = ib;
        win = ib + 8;
        wincol = win + kMaxD;
        cg_active = wincol + kMaxD;
        cg_any = cg_active + kMaxD;
        tickets = reinterpret_cast<unsigned*>(cg_any + 8);
        napplies = reinterpret_cast<unsigned long long*>(tickets + 8);
        CK(hipMemsetAsync(ismall.p, 0, ismall.bytes, st));
        CK(hipHostMalloc((void**)&hs, sizeof(HostStatus), hipHostMallocDefault));
        CK(hipEventCreateWithFlags(&np_ev, hipEventDisableTiming));
        if (batch) {
            CK(hipEventCreateWithFlags(&ev_ready, hipEventDisableTiming));
            CK(hipEventCreateWithFlags(&ev_done, hipEventDisableTiming));
        }
        CK(hipHostMalloc((void**)&note_h, sizeof(unsigned long long), hipHostMallocMapped | hipHostMallocCoherent));
        *note_h = 0;
        CK(hipHostGetDevicePointer((void**)&note_d, note_h, 0));
        return LREP_OK;
    }

    CgState cg_state(int idx_ticket, int which) {
        CgState s;
        s.X = cgX.p;
        s.R = cgR.p;
        s.P = cgP.p;
        s.Q = cgQ.p;
        s.rr = cg_rr;
        s.bb = cg_bb;
        s.alpha = cg_alpha;
        s.beta = cg_beta;
        s.active = cg_active;
        s.any_active = cg_any;
        s.part = part;
        s.part_elems = (size_t)256 * kMaxD * 4;
        s.ticket = tickets + idx_ticket;
        s.napplies = napplies + which;
        s.note = note_d;
        s.seq = ++cg_seq;
        s.c = cg_c;
        s.T = cg_T;
        return s;
    }

    int apply(int which, const double* X, int64_t ldx, int cols, double* Y, int64_t ldy, const int* flag = nullptr,
              hipEvent_t* ev = nullptr, double* pq = nullptr) {
        return op_apply(op, st, which, X, ldx, cols, Y, ldy, gwork.p, GEMM_WORK_ELEMS, Tlr, flag, ev, pq);
    }

    // the dense operator for the fused CG path (nullptr: use the generic apply)
    const double* cg_stream_operator(int which, int nw) const {
        if (op->kind != 0 || nw > 32) return nullptr;
        const bool useK = (which == 0) != op->null_on_M();
        const double* Ad = useK ? op->K : op->M;
        if ((op->ld % 2) != 0 || (reinterpret_cast<uintptr_t>(Ad) % 16) != 0) return nullptr;
        return Ad;
    }

    // low-rank operators: the fused CG (one pass over the rows per step, L
    // read once): 1 for the diagonal operator, 2 for diag + 2 L L^T, else 0
    int fused_cg_kind(int which, int nw) const {
        if (op->kind != 1 || nw < 1 || nw > 32 || n < 64 || (n & 1) || o.fused_cg < 0 ||
            (reinterpret_cast<uintptr_t>(op->delta) & 15))
            return 0;
        const bool useK = (which == 0) != op->null_on_M();
        if (useK) return 1;
        if (!op->Lr || op->rank > 256 || (reinterpret_cast<uintptr_t>(op->Lr) & 15)) return 0;
        return 2;
    }

    // fused CG on a low-rank operator (see fused_cg_kind)
    int cg_fused(int kind, int which, const double* B, int64_t ldb, int nw, double cgtol, int maxit) {
        CgState s = cg_state(1, which);
        const double* Lr = kind == 2 ? op->Lr : nullptr;
        const int r = kind == 2 ? (int)op->rank : 0;
        CK(fused_cg_init(st, (int)n, r, nw, op->delta, Lr, s, B, ldb, cgtol, gwork.p, GEMM_WORK_ELEMS));
        for (int it = 0; it < maxit; ++it) {
            if (it > 0 && !capturing) {
                const unsigned long long v = __atomic_load_n(note_h, __ATOMIC_ACQUIRE);
                if ((v >> 1) == s.seq && (v & 1ull) == 0) break;
            }
            int* logslot = nullptr;
            hipEvent_t* ev = (o.profile && kind == 2) ? prof_next(nw, &logslot, 0, true) : nullptr;
            CK(fused_cg_step(st, (int)n, r, nw, op->delta, Lr, s, cgtol, gwork.p, GEMM_WORK_ELEMS, ev, logslot,
                             kind == 2 && o.precision == 4 ? op->Lr32() : nullptr));
        }
        return LREP_OK;
    }

    // solution of A x_j = rhs_j (which: 0 = K, 1 = M; B with ld ldb) into cgX
    // (ld n); `maxit` CG steps
    int cg(int which, const double* B, int64_t ldb, int nw, double cgtol, int maxit, bool host_check) {
        // the long, tight-tolerance CG of the null-space set-up keeps the plain form
        if (const int fk = host_check ? 0 : fused_cg_kind(which, nw))
            return cg_fused(fk, which, B, ldb, nw, cgtol, maxit);
        CgState s = cg_state(1, which);
        CK(cg_init(st, (int)n, nw, s, B, ldb, cgtol));
        const double* Ad = cg_stream_operator(which, nw);
        const int ntiles = (int)stream_tiles((int)n);
        // low-rank operators: the apply also returns p.q per 64-row tile
        const bool lr_pq = !Ad && op_apply_has_pq(op, which, cgP.p, n, nw);
        const bool lr_diag = lr_pq && ((which == 0) != op->null_on_M());   // K = diag(delta)
        // mixed precision: the product on the 16-bit operator copy
        const uint16_t* A16 = nullptr;
        if (Ad && o.precision != 0 && op->prec16 == o.precision) {
            const bool useK = (which == 0) != op->null_on_M();
            A16 = useK ? op->K16() : op->M16();
        }
        for (int it = 0; it < maxit; ++it) {
            // the device posts "no column active" for this solve: every step
            // not yet issued would return at once, so stop issuing them
            if (it > 0 && !capturing) {
                const unsigned long long v = __atomic_load_n(note_h, __ATOMIC_ACQUIRE);
                if ((v >> 1) == s.seq && (v & 1ull) == 0) break;
            }
            int* logslot = nullptr;
            // timed: the dense applies, and the low-rank M applies (the K applies of
            // the low-rank operator are a diagonal scaling)
            const bool timed =
                o.profile && (op->kind == 0 || (op->kind == 1 && ((which == 0) == op->null_on_M())));
            hipEvent_t* ev = timed ? prof_next(nw, Ad ? &logslot : nullptr, A16 ? o.precision : 0) : nullptr;
            if (A16) {
                CK(cg_dense_apply16(st, o.precision, (int)n, nw, A16, cgP.p, cgR.p, cg_beta, cg_active, cg_rr,
                                    it == 0 ? 1 : 0, cgQ.p, cg_pq, gwork.p, GEMM_WORK_ELEMS, cg_any, ev, logslot));
                CK(cg_update_tiles(st, (int)n, nw, ntiles, cg_pq, s, cgtol));
            } else if (Ad) {
                // direction update of the previous step, pack, apply, p.q per tile
                CK(cg_dense_apply(st, (int)n, nw, Ad, op->ld, cgP.p, cgR.p, cg_beta, cg_active, it == 0 ? 1 : 0,
                                  cgQ.p, cg_pq, gwork.p, GEMM_WORK_ELEMS, cg_any, ev, logslot));
                CK(cg_update_tiles(st, (int)n, nw, ntiles, cg_pq, s, cgtol));
            } else if (lr_diag) {
                // diagonal K of a low-rank operator: the direction update of the
                // previous step is folded into this step's apply
                if (it == 0)
                    CK(diag_scale_pq(st, (int)n, nw, op->delta, cgP.p, n, cgQ.p, n, cg_pq, cg_any));
                else
                    CK(diag_dir_scale_pq(st, (int)n, nw, op->delta, cgP.p, cgR.p, cg_beta, cg_active, cgQ.p, cg_pq,
                                         cg_any));
                CK(cg_update_tiles(st, (int)n, nw, ntiles, cg_pq, s, cgtol));
            } else if (lr_pq) {
                CR(apply(which, cgP.p, n, nw, cgQ.p, n, cg_any, ev, cg_pq));
                CK(cg_update_tiles(st, (int)n, nw, ntiles, cg_pq, s, cgtol));
                CK(cg_direction(st, (int)n, nw, s));
            } else {
                CR(apply(which, cgP.p, n, nw, cgQ.p, n, cg_any, ev));
                CK(lrep::cg_alpha(st, (int)n, nw, s));
                CK(cg_update(st, (int)n, nw, s, cgtol));
                CK(cg_direction(st, (int)n, nw, s));
            }
            if (host_check && (it % 50 == 49)) {
                int any = 0;
                CK(hipMemcpyAsync(&hs->status[7], cg_any, sizeof(int), hipMemcpyDeviceToHost, st));
                CK(hipStreamSynchronize(st));
                any = hs->status[7];
                if (!any) break;
            }
        }
        return LREP_OK;
    }

    int read_status() {
        CK(hipMemcpyAsync(hs->status, status, sizeof(int) * ST_COUNT, hipMemcpyDeviceToHost, st));
        CK(hipStreamSynchronize(st));
        return LREP_OK;
    }

    // Step-6 CG of a served request, batched with other requests on the same
    // operator (continuous batching of the CG applies).  The job waits in the
    // operator's queue while another batch runs (until the device has finished
    // it); the thread whose job is pending when no batch runs leads the next
    // one: its own job first, then the queued jobs with the same CG settings,
    // up to 32 columns.  The
    // leader gathers the right-hand sides (after each owner's `ready` event),
    // runs one CG on its own stream and CG state, and hands every other job
    // its columns (then `done`).  A thread leads only batches holding its own
    // job, so no leader writes the CG state of a thread that runs anything.
    // Every CG kernel treats the columns independently (the same arithmetic in
    // the same order whatever the block width and position), so each column's
    // result is bitwise the one it has alone.
    int cg_batched(int which, const double* B, int64_t ldb, int nw, double cgtol, int maxit) {
        CgJob job{};
        job.owner = this;
        job.which = which;
        job.nw = nw;
        job.maxit = maxit;
        job.precision = o.precision;
        job.fused = o.fused_cg;
        job.tol = cgtol;
        job.B = B;
        job.ldb = ldb;
        job.X = cgX.p;
        job.ready = ev_ready;
        job.done = ev_done;
        CK(hipEventRecord(ev_ready, st));
        std::unique_lock<std::mutex> lk(op->batch_mu);
        op->batch_queue.push_back(&job);
        while (!job.finished) {
            if (op->batch_running) {
                op->batch_cv.wait(lk);
                continue;
            }
            // lead a batch: this job first, then compatible waiting jobs
            std::vector<CgJob*> grp{&job};
            int total = nw;
            auto& q = op->batch_queue;
            for (auto it = q.begin(); it != q.end();) {
                CgJob* j = *it;
                if (j == &job) {
                    it = q.erase(it);
                } else if (j->compatible(job) && total + j->nw <= 32) {
                    grp.push_back(j);
                    total += j->nw;
                    it = q.erase(it);
                } else {
                    ++it;
                }
            }
            op->batch_running = true;
            lk.unlock();
            int rc = run_batch(grp, total);
            // the batch holds the operator until the device has run it: solves
            // that start meanwhile queue up and form the next batch
            if (rc == LREP_OK) {
                const hipError_t e = hipEventSynchronize(job.done);
                if (e != hipSuccess) rc = dev_fail(e, "hipEventSynchronize(batch done)");
            }
            lk.lock();
            for (CgJob* j : grp) {
                j->rc = rc;
                j->shared = grp.size() > 1;
                j->finished = true;
            }
            op->batch_running = false;
            op->batch_cv.notify_all();
        }
        lk.unlock();
        if (job.shared) stats.cg_batched++;
        if (job.rc != LREP_OK) return job.rc;
        // led by another thread: continue after its hand-over
        CK(hipStreamWaitEvent(st, ev_done, 0));
        return LREP_OK;
    }

    // one block CG over the jobs' columns (grp[0] is this solver's own job)
    int run_batch(const std::vector<CgJob*>& grp, int total) {
        const CgJob& mine = *grp[0];
        if (grp.size() == 1) {
            CR(cg(mine.which, mine.B, mine.ldb, mine.nw, mine.tol, mine.maxit, false));
            CK(hipEventRecord(mine.done, st));
            return LREP_OK;
        }
        int off = 0;
        for (const CgJob* j : grp) {
            if (j->owner != this) CK(hipStreamWaitEvent(st, j->ready, 0));
            CK(copy_cols(st, (int)n, j->nw, j->B, j->ldb, bcomb.p + (size_t)off * n, n));
            off += j->nw;
        }
        CR(cg(mine.which, bcomb.p, n, total, mine.tol, mine.maxit, false));
        off = 0;
        for (const CgJob* j : grp) {
            // this solver's own columns are already in place (offset 0 of cgX)
            if (j->owner != this) {
                CK(copy_cols(st, (int)n, j->nw, cgX.p + (size_t)off * n, n, j->X, n));
                stats.cg_batch_columns += j->nw;
            }
            off += j->nw;
        }
        for (const CgJob* j : grp) CK(hipEventRecord(j->done, st));
        return LREP_OK;
    }

    // Step 6's CG: batched with other served requests where allowed
    int cg_step6(int which, const double* B, int64_t ldb, int nw, double cgtol, int maxit) {
        if (batch && nw <= 32) return cg_batched(which, B, ldb, nw, cgtol, maxit);
        return cg(which, B, ldb, nw, cgtol, maxit, false);
    }

    // Gram C = A^T B for segment lists
    int gram(const std::vector<Seg>& A, const std::vector<Seg>& B, double* C, int64_t ldc, int sym) {
        int p = 0, q = 0;
        for (auto& s : A) p += s.cols;
        for (auto& s : B) q += s.cols;
        if (p == 0 || q == 0) return LREP_OK;
        CK(gemm_tn(st, (int)n, p, q, A.data(), (int)A.size(), B.data(), (int)B.size(), C, ldc, 1.0, sym, gwork.p,
                   GEMM_WORK_ELEMS));
        return LREP_OK;
    }
    // C = alpha A B + beta C, A a segment list (n x p), B p x q (ldb)
    int prod(const std::vector<Seg>& A, const double* B, int64_t ldb, int q, double* C, int64_t ldc, double alpha,
             double beta) {
        int p = 0;
        for (auto& s : A) p += s.cols;
        if (q == 0) return LREP_OK;
        CK(gemm_nn(st, (int)n, q, p, A.data(), (int)A.size(), B, ldb, C, ldc, alpha, beta, gwork.p,
                   GEMM_WORK_ELEMS));
        return LREP_OK;
    }
    static std::vector<Seg> segs(std::initializer_list<Seg> l) {
        std::vector<Seg> v;
        for (auto& s : l)
            if (s.cols > 0) v.push_back(s);
        return v;
    }

    // Block MGS-Biorth of (X, Y) (n x m, ld ldi) into (oX, oY) (ld ldo; may alias X, Y).
    int block_mgs(double* X, double* Y, int64_t ldi, int m, double* oX, double* oY, int64_t ldo, int* kept) {
        *kept = 0;
        if (m == 0) return LREP_OK;
        const int64_t ldg = 2 * kMaxD;
        // pass 1
        CR(gram(segs({{X, ldi, m}, {Y, ldi, m}}), segs({{X, ldi, m}, {Y, ldi, m}}), G, ldg, 0));
        CK(coef_mgs(st, m, G, ldg, Acoef, Bcoef, status, MGS_COS_TOL, MGS_DEP_TOL_COEF, scr));
        CR(read_status());
        const int k1 = hs->status[ST_NKEPT];
        stats.mgs_drops += m - k1;
        if (k1 == 0) return LREP_OK;
        CR(prod(segs({{X, ldi, m}}), Acoef, kMaxD, k1, tX.p, ldn, 1.0, 0.0));
        CR(prod(segs({{Y, ldi, m}}), Bcoef, kMaxD, k1, tY.p, ldn, 1.0, 0.0));
        // pass 2
        CR(gram(segs({{tX.p, ldn, k1}, {tY.p, ldn, k1}}), segs({{tX.p, ldn, k1}, {tY.p, ldn, k1}}), G, ldg, 0));
        CK(coef_mgs(st, k1, G, ldg, Acoef, Bcoef, status, MGS_COS_TOL, MGS_DEP_TOL_COEF, scr));
        CR(read_status());
        const int k2 = hs->status[ST_NKEPT];
        stats.mgs_drops += k1 - k2;
        CR(prod(segs({{tX.p, ldn, k1}}), Acoef, kMaxD, k2, oX, ldo, 1.0, 0.0));
        CR(prod(segs({{tY.p, ldn, k1}}), Bcoef, kMaxD, k2, oY, ldo, 1.0, 0.0));
        *kept = k2;
        return LREP_OK;
    }

    // U <- (I - X0 Y0^T) U, V <- (I - Y0 X0^T) V (U, V with ld ldn; X0, Y0 ld n)
    int project_v0(double* U, double* V, int d) {
        if (r0 == 0 || d == 0) return LREP_OK;
        CR(gram(segs({{op->Y0.p, n, r0}}), segs({{U, ldn, d}}), Cproj, kproj, 0));
        CR(prod(segs({{op->X0.p, n, r0}}), Cproj, kproj, d, U, ldn, -1.0, 1.0));
        CR(gram(segs({{op->X0.p, n, r0}}), segs({{V, ldn, d}}), Cproj, kproj, 0));
        CR(prod(segs({{op->Y0.p, n, r0}}), Cproj, kproj, d, V, ldn, -1.0, 1.0));
        return LREP_OK;
    }

    int run(double* lambda_out, double* X_out, double* Y_out, int64_t ldxy);
};

int Solver::run(double* lambda_out, double* X_out, double* Y_out, int64_t ldxy) {
    auto t0 = std::chrono::steady_clock::now();
    const int d0 = b + 2 * w;
    // Step 6 as a replayed graph (on request only: replays measured no faster
    // than the stream path, whose small launches are bound by the device's
    // kernel-to-kernel latency rather than by the host issuing them); not
    // around a caller's function (it may synchronise) nor with per-launch
    // profiling events
    const bool use_graphs = op->kind != 2 && !o.profile && o.graphs == 1;
    int cur = 0, off = 0;
    int d = d0;
    // phases: 0 initialise U, V / 1 small-scale problem (applies, projection,
    // Ritz pairs, pull-back) / 2 convergence check / 3 P, Q / 4 W, Z
    mark(0);
    // Step 1: starting block, V = U
    double* U0 = bX[0].p;
    double* V0 = bY[0].p;
    if (o.init_U) {
        if (o.init_on_device)
            CK(hipMemcpy2DAsync(U0, ldn * sizeof(double), o.init_U, o.ld_init * sizeof(double), n * sizeof(double),
                                d0, hipMemcpyDeviceToDevice, st));
        else
            CK(hipMemcpy2DAsync(U0, ldn * sizeof(double), o.init_U, o.ld_init * sizeof(double), n * sizeof(double),
                                d0, hipMemcpyHostToDevice, st));
        // with a metric the start block is given in the original coordinates
        for (int c0 = 0; c0 < d0; c0 += kMaxD)
            CR(op_metric_transform(op, st, true, std::min(kMaxD, d0 - c0), U0 + (size_t)c0 * ldn, ldn, tX.p, gwork.p,
                                   GEMM_WORK_ELEMS));
    } else {
        CK(philox_normal(st, (int)n, d0, o.seed, U0, ldn));
    }
    CK(copy_cols(st, (int)n, d0, U0, ldn, V0, ldn));
    // Step 2
    CR(project_v0(U0, V0, d0));
    int kept = 0;
    CR(block_mgs(U0, V0, ldn, d0, U0, V0, ldn, &kept));
    d = kept;
    std::vector<double> lamc;
    int c = 0;
    const int lock_unit = std::min(2 * w, b);
    int it = 0;
    const bool trace = std::getenv("LREP_TRACE") != nullptr;
    bool just_restored = false;
    // K U and M V: applied afresh (need_fresh, or every `interval`
    // iterations) or carried through the basis updates for `carried`
    // iterations.  Each refresh after carried iterations measures how far the
    // carried images drifted from the fresh ones; the interval halves when
    // the drift reaches 1e-2 tol and doubles (up to o.refresh) below 1e-3 tol.
    bool need_fresh = true;
    int carried = 0;
    int interval = std::min(2, o.refresh);
    bool drift_pending = false;
    double last_drift = 0.0;
    int rc = LREP_ENOTCONV;
    std::vector<double> epsc;
    while (it < o.maxit) {
        if (d < 1) return fail(LREP_EBREAKDOWN, "subspace empty after MGS-Biorth");
        ++it;
        const int nxt = 1 - cur;
        double* U = bX[cur].p + (size_t)off * ldn;
        double* V = bY[cur].p + (size_t)off * ldn;
        double* KU = bKX[cur].p + (size_t)off * ldn;
        double* MV = bMY[cur].p + (size_t)off * ldn;
        double* NX = bX[nxt].p;
        double* NY = bY[nxt].p;
        double* NKX = bKX[nxt].p;
        double* NMY = bMY[nxt].p;
        const int need = nev - c;
        // Step 3
        mark(1);
        if (need_fresh || carried >= interval - 1) {
            if (carried > 0 && !need_fresh) {
                CR(apply(0, U, ldn, d, tX.p, ldn));
                CR(apply(1, V, ldn, d, tY.p, ldn));
                CK(image_drift(st, (int)n, d, KU, tX.p, MV, tY.p, ldn, part, (size_t)256 * kMaxD * 4, offmax + 1));
                CK(copy_cols(st, (int)n, d, tX.p, ldn, KU, ldn));
                CK(copy_cols(st, (int)n, d, tY.p, ldn, MV, ldn));
                drift_pending = true;
            } else {
                CR(apply(0, U, ldn, d, KU, ldn));
                CR(apply(1, V, ldn, d, MV, ldn));
            }
            stats.applies_K += d;
            stats.applies_M += d;
            need_fresh = false;
            carried = 0;
        } else {
            ++carried;
        }
        CR(gram(segs({{U, ldn, d}}), segs({{KU, ldn, d}}), Kh, kMaxD, 1));
        CR(gram(segs({{V, ldn, d}}), segs({{MV, ldn, d}}), Mh, kMaxD, 1));
        CR(gram(segs({{U, ldn, d}}), segs({{V, ldn, d}}), S, kMaxD, 0));
        CK(max_offidentity(st, d, S, kMaxD, offmax));
        CK(small_lrep(st, d, Kh, Mh, kMaxD, lam, Xh, Yh, scr, status, gwork.p, GEMM_WORK_ELEMS));
        const int nr = std::min(b, d);
        auto pull = [&](int g0, int g1, int col0) -> int {
            if (g1 <= g0) return LREP_OK;
            const int k = g1 - g0;
            const Seg A4[4] = {{U, ldn, d}, {V, ldn, d}, {KU, ldn, d}, {MV, ldn, d}};
            const double* B4[4] = {Xh + (size_t)g0 * kMaxD, Yh + (size_t)g0 * kMaxD, Xh + (size_t)g0 * kMaxD,
                                   Yh + (size_t)g0 * kMaxD};
            double* C4[4] = {NX + (size_t)col0 * ldn, NY + (size_t)col0 * ldn, NKX + (size_t)col0 * ldn,
                             NMY + (size_t)col0 * ldn};
            CK(gemm_nn_batch(st, (int)n, k, d, 4, A4, B4, kMaxD, C4, ldn, 1.0, 0.0));
            return LREP_OK;
        };
        CR(pull(0, nr, 0));
        // Step 4
        mark(2);
        CK(residual_eps(st, (int)n, nr, NX, NY, NKX, NMY, ldn, lam, eps, part, (size_t)256 * kMaxD * 4, tickets));
        CK(hipMemcpyAsync(hs->eps, eps, sizeof(double) * nr, hipMemcpyDeviceToHost, st));
        CK(hipMemcpyAsync(hs->lam, lam, sizeof(double) * d, hipMemcpyDeviceToHost, st));
        CK(hipMemcpyAsync(&hs->offmax, offmax, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        CR(read_status());
        if (hs->status[ST_NOTSPD]) return fail(LREP_ENOTSPD, "Cholesky of a projected matrix failed");
        if (drift_pending) {
            drift_pending = false;
            last_drift = hs->drift;
            if (!(last_drift < 1e-2 * tol))
                interval = std::max(1, interval / 2);
            else if (last_drift < 1e-3 * tol)
                interval = std::min(o.refresh, 2 * interval);
        }
        if (trace) {
            double em = 0;
            for (int g = 0; g < nr; ++g) em = std::max(em, hs->eps[g]);
            std::fprintf(stderr,
                         "[lrep] it=%d d=%d locked=%d offmax=%.3e max_eps=%.3e lam0=%.15e sweeps=%d carried=%d "
                         "interval=%d drift=%.3e\n",
                         it, d, c, hs->offmax, em, hs->lam[0], hs->status[ST_SWEEPS], carried, interval, last_drift);
        }
        // biorthogonality monitor: restore U^T V = I and redo the iteration (the
        // check is skipped on the pass right after a restore, as the check
        // happens once per iteration before the projection)
        if (!std::isfinite(hs->offmax)) return fail(LREP_ENUMERIC, "non-finite value in U^T V");
        if (!just_restored && !(hs->offmax <= o.rebiorth_tol)) {
            --it;
            stats.rebiorth++;
            just_restored = true;
            if (hs->offmax <= 1e-8) {
                // small loss: first-order correction with S = U^T V,
                // U Bx, V By (Bx = I - (S - I)^T / 2, By = I - (S - I) / 2) and
                // the images with them, so (U Bx)^T (V By) = I + O(|S - I|^2) and
                // K (U Bx) = (K U) Bx stays exact; the corrected basis is
                // written to the other buffer set (free until the pull-back of
                // the redone iteration)
                CK(biorth_fix_coef(st, d, S, kMaxD, Acoef, Bcoef, kMaxD));
                const Seg A4[4] = {{U, ldn, d}, {V, ldn, d}, {KU, ldn, d}, {MV, ldn, d}};
                const double* B4[4] = {Acoef, Bcoef, Acoef, Bcoef};
                double* C4[4] = {NX, NY, NKX, NMY};
                CK(gemm_nn_batch(st, (int)n, d, d, 4, A4, B4, kMaxD, C4, ldn, 1.0, 0.0));
                cur = nxt;
                off = 0;
                continue;
            }
            need_fresh = true;
            CR(block_mgs(U, V, ldn, d, U, V, ldn, &kept));
            d = kept;
            continue;
        }
        just_restored = false;
        for (int g = 0; g < nr; ++g)
            if (!std::isfinite(hs->eps[g]) || !std::isfinite(hs->lam[g]))
                return fail(LREP_ENUMERIC, "non-finite Ritz value or residual");
        int p = 0;
        while (p < nr && hs->eps[p] <= tol) ++p;
        if (carried > 0 && (p >= need || (p >= lock_unit && d > lock_unit))) {
            // pairs are about to be locked or returned: test them on images
            // applied afresh to this subspace
            --it;
            need_fresh = true;
            continue;
        }
        if (p >= need) {
            // converged: X = [Xc, X~(:, 0:need)]
            CK(copy_cols(st, (int)n, need, NX, ldn, Xc.p + (size_t)c * ldn, ldn));
            CK(copy_cols(st, (int)n, need, NY, ldn, Yc.p + (size_t)c * ldn, ldn));
            for (int g = 0; g < need; ++g) {
                lamc.push_back(hs->lam[g]);
                epsc.push_back(hs->eps[g]);
            }
            c += need;
            rc = LREP_OK;
            break;
        }
        int L = (p >= lock_unit && d > lock_unit) ? lock_unit : 0;
        if (L) {
            CK(copy_cols(st, (int)n, L, NX, ldn, Xc.p + (size_t)c * ldn, ldn));
            CK(copy_cols(st, (int)n, L, NY, ldn, Yc.p + (size_t)c * ldn, ldn));
            for (int g = 0; g < L; ++g) {
                lamc.push_back(hs->lam[g]);
                epsc.push_back(hs->eps[g]);
            }
            c += L;
            stats.locks++;
        }
        const int hi = std::min(L + b, d);
        std::vector<int> wg;   // window Ritz indices
        for (int g = L; g < hi && (int)wg.size() < w; ++g)
            if (g >= nr || hs->eps[g] > tol) wg.push_back(g);
        for (int g = hi; g < d && (int)wg.size() < w; ++g) wg.push_back(g);
        // pull back what is not there yet: [nr, hi) at natural columns, extension g >= hi at g + 2w
        mark(1);
        CR(pull(nr, hi, nr));
        {
            // the extension indices are consecutive from hi: one batched pull
            int ext = 0;
            for (int g : wg) ext += g >= hi;
            if (ext > 0) CR(pull(hi, hi + ext, hi + 2 * w));
        }
        const int na = hi - L;
        if (wg.empty()) {
            cur = nxt;
            off = L;
            d = na;
            continue;
        }
        const int nw = (int)wg.size();
        std::vector<int> wcol(nw);
        std::vector<double> lw(nw);
        for (int j = 0; j < nw; ++j) {
            wcol[j] = wg[j] < hi ? wg[j] : wg[j] + 2 * w;
            lw[j] = hs->lam[wg[j]];
        }
        CK(hipMemcpyAsync(win, wg.data(), sizeof(int) * nw, hipMemcpyHostToDevice, st));
        CK(hipMemcpyAsync(wincol, wcol.data(), sizeof(int) * nw, hipMemcpyHostToDevice, st));
        CK(hipMemcpyAsync(lamw, lw.data(), sizeof(double) * nw, hipMemcpyHostToDevice, st));
        // Step 5
        mark(3);
        CK(step5_pq(st, d, hi, Xh, Yh, win, nw, Ph, Qh, scr, status, MGS_COS_TOL, MGS_DEP_TOL, gwork.p, GEMM_WORK_ELEMS));
        // the number np of kept P~ columns is first needed after Step 6's CG
        // (which reads only window columns, below hi or from hi + 2w, and
        // writes only the CG buffers): fetch it behind an event and wait for it
        // while the CG runs, instead of draining the stream here
        CK(hipMemcpyAsync(hs->status, status, sizeof(int) * ST_COUNT, hipMemcpyDeviceToHost, st));
        CK(hipEventRecord(np_ev, st));
        // Step 6: block Gauss-Seidel sweeps with CG
        mark(4);
        auto step6 = [&]() -> int {
            for (int j = 0; j < o.ngs; ++j) {
                CK(gs_rhs(st, (int)n, nw, j == 0 ? nullptr : Ws.p, ldn, NX, NMY, ldn, wincol, lamw, rhs.p, ldn));
                CR(cg_step6(1, rhs.p, ldn, nw, o.cg_tol, o.cg_maxit));
                CK(copy_cols(st, (int)n, nw, cgX.p, n, Zs.p, ldn));
                CK(gs_rhs(st, (int)n, nw, Zs.p, ldn, NY, NKX, ldn, wincol, lamw, rhs.p, ldn));
                CR(cg_step6(0, rhs.p, ldn, nw, o.cg_tol, o.cg_maxit));
                CK(copy_cols(st, (int)n, nw, cgX.p, n, Ws.p, ldn));
            }
            return LREP_OK;
        };
        if (use_graphs) {
            // the launch sequence depends only on nw and on which of the two
            // basis buffers is current: capture it once, replay it after
            hipGraphExec_t ge = nullptr;
            for (auto& g : graphs6)
                if (g.nw == nw && g.nx == NX) ge = g.exec;
            if (!ge) {
                CK(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
                capturing = true;
                const int rc6 = step6();
                capturing = false;
                hipGraph_t gr = nullptr;
                const hipError_t ec = hipStreamEndCapture(st, &gr);
                if (rc6 != LREP_OK) {
                    if (gr) (void)hipGraphDestroy(gr);
                    return rc6;
                }
                CK(ec);
                const hipError_t ei = hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0);
                (void)hipGraphDestroy(gr);
                CK(ei);
                graphs6.push_back({nw, NX, ge});
            }
            CK(hipGraphLaunch(ge, st));
        } else {
            CR(step6());
        }
        CK(hipEventSynchronize(np_ev));
        const int np = hs->status[ST_NP];
        stats.mgs_drops += nw - np;
        double* Pt = NX + (size_t)hi * ldn;
        double* Qt = NY + (size_t)hi * ldn;
        // the next subspace's images are carried whenever carrying is on, also
        // into a refresh, where they are compared with the fresh ones
        const bool carry_next = interval > 1;
        {
            // P~ = U P^, Q~ = V Q^ (Step 5), into columns [hi, hi + np) of the next basis
            const Seg A4[4] = {{U, ldn, d}, {V, ldn, d}, {KU, ldn, d}, {MV, ldn, d}};
            const double* B4[4] = {Ph, Qh, Ph, Qh};
            double* C4[4] = {Pt, Qt, NKX + (size_t)hi * ldn, NMY + (size_t)hi * ldn};
            CK(gemm_nn_batch(st, (int)n, np, d, carry_next ? 4 : 2, A4, B4, kMaxD, C4, ldn, 1.0, 0.0));
        }
        // projection against [X0, Xc, X~_active, P~], applied twice
        const int kact = na + np;
        auto Xall = segs({{op->X0.p, n, (int)r0}, {Xc.p, ldn, c}, {NX + (size_t)L * ldn, ldn, kact}});
        auto Yall = segs({{op->Y0.p, n, (int)r0}, {Yc.p, ldn, c}, {NY + (size_t)L * ldn, ldn, kact}});
        for (int pass = 0; pass < 2; ++pass) {
            CR(gram(Yall, segs({{Ws.p, ldn, nw}}), Cproj, kproj, 0));
            CR(prod(Xall, Cproj, kproj, nw, Ws.p, ldn, -1.0, 1.0));
            CR(gram(Xall, segs({{Zs.p, ldn, nw}}), Cproj, kproj, 0));
            CR(prod(Yall, Cproj, kproj, nw, Zs.p, ldn, -1.0, 1.0));
        }
        // MGS-Biorth of (W~, Z~), appended after P~
        int nwk = 0;
        CR(block_mgs(Ws.p, Zs.p, ldn, nw, NX + (size_t)(hi + np) * ldn, NY + (size_t)(hi + np) * ldn, ldn, &nwk));
        if (carry_next && nwk > 0) {
            const size_t o2 = (size_t)(hi + np) * ldn;
            CR(apply(0, NX + o2, ldn, nwk, NKX + o2, ldn));
            CR(apply(1, NY + o2, ldn, nwk, NMY + o2, ldn));
            stats.applies_K += nwk;
            stats.applies_M += nwk;
        }
        // Step 7
        cur = nxt;
        off = L;
        d = na + np + nwk;
    }
    // outputs
    CK(hipMemcpyAsync(&hs->napplies[0], napplies, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    stats.applies_K += (int64_t)hs->napplies[0];
    stats.applies_M += (int64_t)hs->napplies[1];
    stats.iterations = it;
    stats.n_converged = c;
    mark(-1);
    if (o.profile) {
        CR(prof_collect());
        CR(collect_phases());
    }
    double me = 0;
    for (double e : epsc) me = std::max(me, e);
    stats.max_eps = me;
    // Pairs of nonzero eigenvalues are biorthogonal to the generalized null
    // space (Lemma 2.3 (iii)); the returned ones only to the rounding level of
    // the bases they were locked from, amplified by the pull-back coefficients.
    // One more projection, a no-op for exact eigenvectors, restores it.
    for (int c0 = 0; c0 < c && r0 > 0; c0 += kMaxD)
        CR(project_v0(Xc.p + (size_t)c0 * ldn, Yc.p + (size_t)c0 * ldn, std::min(kMaxD, c - c0)));
    if (c > 0 && c <= kMaxD) {
        // The returned pairs were locked from bases biorthogonal to the
        // restore threshold; a first-order correction brings X^T Y = I to
        // rounding level (each vector moves by O(|X^T Y - I|), far below the
        // residual tolerance).
        const int64_t ldg = 2 * kMaxD;
        CR(gram(segs({{Xc.p, ldn, c}}), segs({{Yc.p, ldn, c}}), G, ldg, 0));
        CK(biorth_fix_coef(st, c, G, ldg, Acoef, Bcoef, kMaxD));
        const Seg A2[2] = {{Xc.p, ldn, c}, {Yc.p, ldn, c}};
        const double* B2[2] = {Acoef, Bcoef};
        double* C2[2] = {tX.p, tY.p};
        CK(gemm_nn_batch(st, (int)n, c, c, 2, A2, B2, kMaxD, C2, ldn, 1.0, 0.0));
        CK(copy_cols(st, (int)n, c, tX.p, ldn, Xc.p, ldn));
        CK(copy_cols(st, (int)n, c, tY.p, ldn, Yc.p, ldn));
    }
    if (c > 0) {
        double* OX = op->null_on_M() ? Yc.p : Xc.p;
        double* OY = op->null_on_M() ? Xc.p : Yc.p;
        // with a metric B = C C^T, back to the original coordinates: x = C^-T x^, y = C^-T y^
        for (int c0 = 0; c0 < c && op->has_metric(); c0 += kMaxD) {
            const int cc = std::min(kMaxD, c - c0);
            CR(op_metric_transform(op, st, false, cc, OX + (size_t)c0 * ldn, ldn, tX.p, gwork.p, GEMM_WORK_ELEMS));
            CR(op_metric_transform(op, st, false, cc, OY + (size_t)c0 * ldn, ldn, tX.p, gwork.p, GEMM_WORK_ELEMS));
        }
        CK(sign_normalise(st, (int)n, c, OX, OY, ldn));
        const hipMemcpyKind kind = o.result_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
        CK(hipMemcpy2DAsync(X_out, ldxy * sizeof(double), OX, ldn * sizeof(double), n * sizeof(double), c, kind, st));
        CK(hipMemcpy2DAsync(Y_out, ldxy * sizeof(double), OY, ldn * sizeof(double), n * sizeof(double), c, kind, st));
        CK(hipMemcpyAsync(lambda_out, lamc.data(), sizeof(double) * c,
                          o.result_on_device ? hipMemcpyHostToDevice : hipMemcpyHostToHost, st));
        CK(hipStreamSynchronize(st));
    }
    auto t1 = std::chrono::steady_clock::now();
    stats.time_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    if (rc == LREP_ENOTCONV) err = "maximum number of iterations reached";
    return rc;
}

}  // namespace

namespace {
bool lowrank_rows_ok(const Op* op, const double* X, int64_t ldx) {
    return op->Lr && (ldx % 2) == 0 && (reinterpret_cast<uintptr_t>(X) % 16) == 0;
}
}  // namespace

bool op_apply_has_pq(const Op* op, int which, const double* X, int64_t ldx, int cols) {
    if (op->kind != 1 || cols > 32) return false;
    const bool useK = (which == 0) != op->null_on_M();
    return useK || lowrank_rows_ok(op, X, ldx);
}

int op_apply(Op* op, hipStream_t st, int which, const double* X, int64_t ldx, int cols, double* Y, int64_t ldy,
             double* work, size_t work_elems, double* small, const int* active_flag, hipEvent_t* ev, double* pq) {
    if (cols <= 0) return LREP_OK;
    const bool useK = (which == 0) != op->null_on_M();
    hipError_t e = hipSuccess;
    if (pq) {
        if (!op_apply_has_pq(op, which, X, ldx, cols)) return LREP_EINVAL;
        e = useK ? diag_scale_pq(st, (int)op->n, cols, op->delta, X, ldx, Y, ldy, pq, active_flag)
                 : lowrank_apply_M_rows(st, (int)op->n, (int)op->rank, cols, op->delta, op->Lr, X, ldx, Y, ldy, work,
                                        work_elems, active_flag, ev, pq);
        return e == hipSuccess ? LREP_OK : LREP_EDEVICE;
    }
    if (op->kind == 2) {
        const int rc = op->apply_fn(op->apply_user, useK ? 0 : 1, cols, X, ldx, Y, ldy, st);
        if (rc != 0) {
            op->ctx->set_error("operator apply callback returned " + std::to_string(rc));
            return LREP_EDEVICE;
        }
        return LREP_OK;
    }
    if (op->kind == 0) {
        const double* Ad = useK ? op->K : op->M;
        const bool stream_ok = cols <= 32 && (op->ld % 2) == 0 && (reinterpret_cast<uintptr_t>(Ad) % 16) == 0;
        if (stream_ok) {
            e = dense_apply_narrow(st, (int)op->n, cols, (int)op->n, Ad, op->ld, X, ldx, Y, ldy, 1.0, 0.0, work,
                                   work_elems, active_flag, ev);
        } else {
            Seg A{Ad, op->ld, (int)op->n};
            e = gemm_nn(st, (int)op->n, cols, (int)op->n, &A, 1, X, ldx, Y, ldy, 1.0, 0.0, work, work_elems,
                        nullptr, nullptr, 0, 0, active_flag, ev);
        }
    } else if (useK) {
        e = diag_scale(st, (int)op->n, cols, op->delta, X, ldx, Y, ldy, active_flag);
    } else if (lowrank_rows_ok(op, X, ldx)) {
        // streaming low-rank apply on the row-major copy, 32 columns at a time
        for (int c0 = 0; c0 < cols && e == hipSuccess; c0 += 32) {
            const int w = std::min(32, cols - c0);
            e = lowrank_apply_M_rows(st, (int)op->n, (int)op->rank, w, op->delta, op->Lr, X + (size_t)c0 * ldx, ldx,
                                     Y + (size_t)c0 * ldy, ldy, work, work_elems, active_flag,
                                     c0 == 0 ? ev : nullptr);
        }
    } else if (op->rank <= 256 && (op->ldl % 2) == 0 && (ldx % 2) == 0 &&
               (reinterpret_cast<uintptr_t>(op->L) % 16) == 0 && (reinterpret_cast<uintptr_t>(X) % 16) == 0) {
        // streaming low-rank apply, 32 columns at a time
        for (int c0 = 0; c0 < cols && e == hipSuccess; c0 += 32) {
            const int w = std::min(32, cols - c0);
            e = lowrank_apply_M(st, (int)op->n, (int)op->rank, w, op->delta, op->L, op->ldl, X + (size_t)c0 * ldx,
                                ldx, Y + (size_t)c0 * ldy, ldy, work, work_elems, active_flag,
                                c0 == 0 ? ev : nullptr);
        }
    } else {
        Seg Ls{op->L, op->ldl, (int)op->rank};
        Seg Xs{X, ldx, cols};
        e = gemm_tn(st, (int)op->n, (int)op->rank, cols, &Ls, 1, &Xs, 1, small, op->rank, 1.0, 0, work, work_elems,
                    active_flag);
        if (e == hipSuccess)
            e = gemm_nn(st, (int)op->n, cols, (int)op->rank, &Ls, 1, small, op->rank, Y, ldy, 2.0, 0.0, work,
                        work_elems, op->delta, X, ldx, 0, active_flag);
    }
    return e == hipSuccess ? LREP_OK : LREP_EDEVICE;
}

namespace {
// the options with their defaults filled in; LREP_EINVAL for values out of range
int solve_options(const lrep_solve_opts_t* opts, int64_t block, lrep_solve_opts_t& o) {
    o = lrep_solve_opts_t{};
    if (opts) o = *opts;
    if (o.window <= 0) o.window = block;
    if (o.maxit <= 0) o.maxit = 1000;
    if (o.ngs <= 0) o.ngs = 1;
    if (o.cg_maxit <= 0) o.cg_maxit = 20;
    if (!(o.cg_tol > 0)) o.cg_tol = 1e-2;
    if (!(o.rebiorth_tol > 0)) o.rebiorth_tol = 1e-12;
    if (o.refresh <= 0) o.refresh = 8;
    if (o.graphs < -1 || o.graphs > 1 || o.precision < 0 || o.precision > 4 || o.fused_cg < -1 || o.fused_cg > 1 ||
        o.serve_batch < -1 || o.serve_batch > 0)
        return LREP_EINVAL;
    return LREP_OK;
}

// the solver's shape from the arguments (no device work); LREP_EINVAL for sizes out of range
int solve_configure(Solver& s, Op* op, hipStream_t st, int64_t nev, int64_t block, double tol,
                    const lrep_solve_opts_t& o, bool served = false) {
    s.op = op;
    s.st = st;
    s.n = op->n;
    // served solves on dense or low-rank operators may batch their Step-6 CG
    // with other requests' (not under graph capture or per-launch profiling)
    s.batch = served && o.serve_batch == 0 && (op->kind == 0 || op->kind == 1) && o.graphs != 1 && !o.profile &&
              o.window <= 32;
    if (o.precision >= 1 && o.precision <= 3 && op->kind == 0 && (op->n % 8 != 0 || op->n < 64)) return LREP_EINVAL;
    // FP32 rows of L for the fused CG passes: low-rank operators with L only
    if (o.precision == 4 && (op->kind != 1 || !op->Lr)) return LREP_EINVAL;
    if (o.init_U && o.ld_init < op->n) return LREP_EINVAL;
    s.o = o;
    s.b = (int)block;
    s.w = (int)o.window;
    s.nev = (int)nev;
    s.r0 = (int)op->r0;
    s.tol = tol;
    s.cap = s.b + 4 * s.w + 1;
    const int64_t d0 = block + 2 * o.window;
    if (nev < 1 || block < 1 || nev > op->n - op->r0 || d0 > op->n - op->r0 || d0 > kMaxD || s.w > 64 ||
        !(tol > 0))
        return LREP_EINVAL;
    return LREP_OK;
}
}  // namespace

int solve_footprint(Op* op, int64_t nev, int64_t block, double tol, const lrep_solve_opts_t* opts, size_t* bytes,
                    bool served) {
    lrep_solve_opts_t o;
    CR(solve_options(opts, block, o));
    Solver s;
    CR(solve_configure(s, op, nullptr, nev, block, tol, o, served));
    size_t total = s.footprint();
    if (o.precision != 0 && op->kind == 0) {
        std::lock_guard<std::mutex> g(op->mu16);
        if (op->prec16 != o.precision)
            total += 2 * (size_t)(o.precision == 3 ? 3 : 1) * op->n * op->n * sizeof(uint16_t);
    }
    if (o.precision == 4) {
        std::lock_guard<std::mutex> g(op->mu16);
        if (!op->Lr32buf.p) total += (size_t)op->n * lowrank_row_ld(op->rank) * sizeof(float);
    }
    *bytes = total;
    return LREP_OK;
}

int solve(Op* op, hipStream_t st, int64_t nev, int64_t block, double tol, const lrep_solve_opts_t* opts,
          double* lambda, double* X, double* Y, int64_t ldxy, lrep_stats_t* stats) {
    lrep_solve_opts_t o;
    CR(solve_options(opts, block, o));
    Solver s;
    CR(solve_configure(s, op, st, nev, block, tol, o, t_serving));
    if (ldxy < op->n || !lambda || !X || !Y) return LREP_EINVAL;
    if (o.precision != 0 && op->kind == 0) {
        // 16-bit copies of K and M for the mixed-precision CG applies
        std::lock_guard<std::mutex> g(op->mu16);
        if (op->prec16 != o.precision) {
            op->K16buf.release();
            op->M16buf.release();
            op->prec16 = 0;
            const size_t bytes = (size_t)(o.precision == 3 ? 3 : 1) * op->n * op->n * sizeof(uint16_t);
            int rc = op->K16buf.alloc(op->ctx, bytes);
            if (rc == LREP_OK) rc = op->M16buf.alloc(op->ctx, bytes);
            if (rc != LREP_OK) return rc;
            hipError_t e = convert_operator16(st, o.precision, (int)op->n, op->K, op->ld,
                                              reinterpret_cast<uint16_t*>(op->K16buf.p));
            if (e == hipSuccess)
                e = convert_operator16(st, o.precision, (int)op->n, op->M, op->ld,
                                       reinterpret_cast<uint16_t*>(op->M16buf.p));
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) {
                op->ctx->set_error(hipGetErrorString(e));
                return LREP_EDEVICE;
            }
            op->prec16 = o.precision;
        }
    }
    if (o.precision == 4) {
        // FP32 rows of L for the fused CG passes
        std::lock_guard<std::mutex> g(op->mu16);
        if (!op->Lr32buf.p) {
            const int64_t ldr = lowrank_row_ld(op->rank);
            int rc = op->Lr32buf.alloc(op->ctx, (size_t)op->n * ldr * sizeof(float));
            if (rc != LREP_OK) return rc;
            hipError_t e = lowrank_rows_f32(st, (int)op->n, (int)op->rank, op->Lr, const_cast<float*>(op->Lr32()));
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) {
                op->Lr32buf.release();
                op->ctx->set_error(hipGetErrorString(e));
                return LREP_EDEVICE;
            }
        }
    }
    int rc = s.alloc();
    if (rc == LREP_OK) rc = s.run(lambda, X, Y, ldxy);
    if (rc != LREP_OK && !s.err.empty()) op->ctx->set_error(s.err);
    if (stats) *stats = s.stats;
    return rc;
}

int prepare_nullspace(Op* op, hipStream_t st, int64_t r, const double* X0t) {
    // Y0~ = M^-1 X0~ by CG to high accuracy, then (X0, Y0) = MGS-Biorth(X0~, Y0~):
    // with X0~^T Y0~ = Y0~^T M Y0~ SPD the recurrence reduces to X0~ C^-1, Y0~ C^-1
    // with C^T C = X0~^T Y0~ (the equation for the V0 basis).
    Solver s;
    s.op = op;
    s.st = st;
    s.n = op->n;
    s.b = (int)r;
    s.w = (int)r;
    s.cap = 1;
    s.nev = 1;
    s.r0 = 0;
    if (r > kMaxD || r > 64) return LREP_EINVAL;
    int rc = s.alloc();
    if (rc != LREP_OK) return rc;
    Ctx* c = op->ctx;
    rc = op->X0.alloc(c, (size_t)op->n * r * sizeof(double));
    if (rc == LREP_OK) rc = op->Y0.alloc(c, (size_t)op->n * r * sizeof(double));
    if (rc != LREP_OK) return rc;
    const int maxit = (int)std::min<int64_t>(20 * op->n + 100, 200000);
    rc = s.cg(1, X0t, op->n, (int)r, 1e-14, maxit, true);
    if (rc != LREP_OK) return rc;
    int kept = 0;
    rc = s.block_mgs(const_cast<double*>(X0t), s.cgX.p, op->n, (int)r, op->X0.p, op->Y0.p, op->n, &kept);
    if (rc != LREP_OK) return rc;
    if (hipStreamSynchronize(st) != hipSuccess) return LREP_EDEVICE;
    if (kept != r) return LREP_ENOTSPD;
    op->r0 = r;
    return LREP_OK;
}

int find_nullspace(Op* op, hipStream_t st, int64_t rmax, double tol, uint64_t seed, int64_t* r_out,
                   double* res_out) {
    // N(A) of the symmetric positive semidefinite operator A (K, or M with the
    // roles exchanged) by projecting random vectors (the remark on computing the
    // generalized null space asks for the zero eigenvectors of A from a
    // symmetric solver; this is the Krylov route to the same subspace).  CG on
    // A x = A x0 from a zero start keeps its iterates in range(A) and converges
    // to the range component of x0, so z = x0 - x is x0's component in N(A).
    // The CG residual is A z itself.  Projections of rmax random vectors span
    // N(A) when rmax >= dim N(A); block MGS (MGS-Biorth of (Z, Z)) orthonormalises
    // them and drops those dependent on earlier ones.
    if (rmax < 1 || rmax > 64 || rmax >= op->n || !(tol > 0)) return LREP_EINVAL;
    Solver s;
    s.op = op;
    s.st = st;
    s.n = op->n;
    s.b = (int)rmax;
    s.w = (int)rmax;
    s.cap = 1;
    s.nev = 1;
    s.r0 = 0;
    int rc = s.alloc();
    if (rc != LREP_OK) return rc;
    auto dev_fail = [&](hipError_t e, const char* what) { return s.dev_fail(e, what); };
    const int n = (int)op->n, m = (int)rmax;
    double* X0 = s.Ws.p;
    double* Bv = s.rhs.p;
    double* Z = s.Zs.p;
    const int64_t ldg = 2 * kMaxD;
    std::vector<double> gh((size_t)m * m);
    // squared column norms of an n x k block (Gram diagonal)
    auto sqnorms = [&](const double* A, int k, std::vector<double>& out) -> int {
        CR(s.gram(s.segs({{A, (int64_t)n, k}}), s.segs({{A, (int64_t)n, k}}), s.G, ldg, 1));
        CK(hipMemcpy2DAsync(gh.data(), (size_t)k * sizeof(double), s.G, ldg * sizeof(double), (size_t)k * sizeof(double),
                            k, hipMemcpyDeviceToHost, st));
        CK(hipStreamSynchronize(st));
        out.resize(k);
        for (int j = 0; j < k; ++j) out[j] = gh[(size_t)j * k + j];
        return LREP_OK;
    };
    CK(philox_normal(st, n, m, seed, X0, n));
    CR(s.apply(0, X0, n, m, Bv, n));
    std::vector<double> nx, nb, nz, nr;
    CR(sqnorms(X0, m, nx));
    CR(sqnorms(Bv, m, nb));
    double normest = 0.0;   // max ||A x0|| / ||x0||, a lower estimate of ||A||_2
    for (int j = 0; j < m; ++j) normest = std::max(normest, std::sqrt(nb[j] / nx[j]));
    if (!(normest > 0) || !std::isfinite(normest)) {
        op->ctx->set_error("find_nullspace: the semidefinite operator is zero or not finite");
        return LREP_ENUMERIC;
    }
    const int maxit = (int)std::min<int64_t>(20 * (int64_t)n + 100, 200000);
    CR(s.cg(0, Bv, n, m, 1e-15, maxit, true));
    CK(sub_cols(st, n, m, X0, n, s.cgX.p, n, Z, n));
    CR(sqnorms(Z, m, nz));
    // a projection at rounding level carries no null direction (A definite on it)
    int k = 0;
    for (int j = 0; j < m; ++j)
        if (std::sqrt(nz[j]) > 1e-8 * std::sqrt(nx[j])) CK(copy_cols(st, n, 1, Z + (size_t)j * n, n, Bv + (size_t)(k++) * n, n));
    op->r0 = 0;
    op->X0.release();
    op->Y0.release();
    *r_out = 0;
    *res_out = 0.0;
    if (k == 0) return LREP_OK;
    CK(copy_cols(st, n, k, Bv, n, X0, n));
    int kept = 0;
    CR(s.block_mgs(Bv, X0, n, k, Bv, X0, n, &kept));
    if (kept == 0) return LREP_OK;
    // the orthonormal basis must satisfy ||A z|| <= tol ||A||
    CR(s.apply(0, Bv, n, kept, Z, n));
    CR(sqnorms(Z, kept, nr));
    double worst = 0.0;
    for (int j = 0; j < kept; ++j) worst = std::max(worst, std::sqrt(nr[j]) / normest);
    *res_out = worst;
    if (!(worst <= tol)) {
        op->ctx->set_error("find_nullspace: the null-space basis reached ||A z|| / ||A|| = " + std::to_string(worst));
        return LREP_ENOTCONV;
    }
    rc = prepare_nullspace(op, st, kept, Bv);
    if (rc != LREP_OK) {
        op->r0 = 0;
        op->X0.release();
        op->Y0.release();
        return rc;
    }
    *r_out = kept;
    return LREP_OK;
}

}  // namespace lrep

namespace lrep {
// Block MGS-Biorth of (X, Y) in place, for the kernel tests.
int block_mgs_standalone(Ctx* c, hipStream_t st, int64_t n, int m, double* X, double* Y, int* kept) {
    Op op;
    op.ctx = c;
    op.n = n;
    Solver s;
    s.op = &op;
    s.st = st;
    s.n = n;
    s.b = 1;
    s.w = 1;
    s.cap = 1;
    s.nev = 1;
    s.r0 = 0;
    if (m < 0 || m > kMaxD) return LREP_EINVAL;
    int rc = s.alloc();
    if (rc == LREP_OK) rc = s.block_mgs(X, Y, n, m, X, Y, n, kept);
    if (rc == LREP_OK && hipStreamSynchronize(st) != hipSuccess) rc = LREP_EDEVICE;
    return rc;
}

// One Step-6 CG solve (which: 0 = K, 1 = M) of nw <= 32 columns B (ld n) into
// X (ld n), as the solver runs it; fused selects the fused low-rank CG
// (1), the plain CG (-1) or the solver's choice (0).  *applies: column
// applies made.  For the kernel tests.
int cg_standalone(Op* op, hipStream_t st, int which, int nw, const double* B, double* X, double tol, int maxit,
                  int fused, int64_t* applies) {
    Solver s;
    s.op = op;
    s.st = st;
    s.n = op->n;
    s.b = nw;
    s.w = nw;
    s.cap = nw;
    s.nev = 1;
    s.r0 = 0;
    s.o.fused_cg = fused;
    if (nw < 1 || nw > 32 || maxit < 1 || !(tol > 0)) return LREP_EINVAL;
    int rc = s.alloc();
    if (rc == LREP_OK) rc = s.cg(which, B, op->n, nw, tol, maxit, false);
    if (rc == LREP_OK && hipMemcpy2DAsync(X, op->n * sizeof(double), s.cgX.p, op->n * sizeof(double),
                                          op->n * sizeof(double), nw, hipMemcpyDeviceToDevice, st) != hipSuccess)
        rc = LREP_EDEVICE;
    unsigned long long na[2] = {0, 0};
    if (rc == LREP_OK && hipMemcpyAsync(na, s.napplies, sizeof(na), hipMemcpyDeviceToHost, st) != hipSuccess)
        rc = LREP_EDEVICE;
    if (rc == LREP_OK && hipStreamSynchronize(st) != hipSuccess) rc = LREP_EDEVICE;
    if (applies) *applies = (int64_t)(na[0] + na[1]);
    return rc;
}
}  // namespace lrep
