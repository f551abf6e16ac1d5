// Allocation-free operator apply (lrep_apply_noalloc).
//
// The same products as lrep_test_apply (Y = K X or Y = M X on device blocks),
// with every intermediate of the kernels -- the k-major packed block and the
// split-k partial tiles of the dense streaming apply, the chunk partials and
// L^T X of the low-rank passes, the split partials of the tall-skinny
// products -- carved from one fixed device array instead of workspaces
// allocated per call.  For callers that cannot allocate device memory (code
// under HIP graph capture, tight serving loops, harnesses that forbid it).
//
// The array lives in the library's code object: each device holds its own
// copy, at its own address, from the first use of the library on that device
// until the process ends.  Host code never passes the array's name to a
// kernel (on the host it is only a stand-in for the symbol): lrep_init looks
// up the device address once per device with hipGetSymbolAddress and every
// call uses that pointer.  Every call on a device shares the device's array,
// so calls that overlap on one device (two streams, two contexts) race; the
// kernels write every element they read, so nothing needs clearing.
#include <mutex>

#include "internal.hpp"
#include "kernels.hpp"

namespace lrep {

namespace {

// 4.5 Mi doubles for the kernels' work area, 0.5 Mi for L^T X of the
// general low-rank product: 40 MiB in all
constexpr size_t kWorkElems = size_t(9) << 19;
constexpr size_t kSmallElems = size_t(1) << 19;
constexpr int kMaxDevices = 64;

__device__ __align__(256) double scratch[kWorkElems + kSmallElems];

std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};

}  // namespace

// device address of this device's scratch array (called by lrep_init with
// the device current); LREP_OK or LREP_EDEVICE
int noalloc_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return LREP_EDEVICE;
    std::lock_guard<std::mutex> g(g_mu);
    if (g_ptr[device]) return LREP_OK;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return LREP_EDEVICE;
    g_ptr[device] = static_cast<double*>(p);
    return LREP_OK;
}

static double* noalloc_ptr(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> g(g_mu);
    return g_ptr[device];
}

}  // namespace lrep

using namespace lrep;
struct lrep_ctx_s : public Ctx {};
struct lrep_op_s : public Op {};

extern "C" int lrep_apply_noalloc(lrep_op_t op, int which, int cols, const double* X, double* Y) {
    if (!op || cols < 0 || (which != 0 && which != 1) || (cols > 0 && (!X || !Y))) return LREP_EINVAL;
    Ctx* c = op->ctx;
    if (hipSetDevice(c->device) != hipSuccess) return LREP_EDEVICE;
    double* s = noalloc_ptr(c->device);
    if (!s) {
        c->set_error("lrep_apply_noalloc: no scratch address for this device");
        return LREP_EDEVICE;
    }
    if (cols == 0) return LREP_OK;
    // what the fixed array holds: the dense streaming apply (<= 32 columns)
    // needs 64 n doubles; the general low-rank product rank x cols for L^T X
    const bool useK = (which == 0) != op->null_on_M();
    if (op->kind == 0 && cols <= 32 && (size_t)op->n * 64 > kWorkElems) {
        c->set_error("lrep_apply_noalloc: dense operators are limited to n <= 73728 (fixed 36 MiB work area)");
        return LREP_EINVAL;
    }
    if (op->kind == 1 && !useK && (size_t)op->rank * (size_t)cols > kSmallElems) {
        c->set_error("lrep_apply_noalloc: rank x cols must not exceed 524288 (fixed 4 MiB area for L^T X)");
        return LREP_EINVAL;
    }
    int rc = op_apply(op, c->stream, which, X, op->n, cols, Y, op->n, s, kWorkElems, s + kWorkElems, nullptr);
    if (rc != LREP_OK) return rc;
    const hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        c->set_error(hipGetErrorString(e));
        return LREP_EDEVICE;
    }
    return LREP_OK;
}
