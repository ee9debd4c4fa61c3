// Operator application whose workspace is a fixed static device array instead
// of the plan's workspace: for callers that cannot allocate (code under graph
// capture, serving loops that forbid allocation).  The kernels are the ones
// toeplitz_matvec launches; only the addresses of the transform grids, the rim
// slab partials and the mirror parts differ.
#include <mutex>
#include <string>

#include "tp_internal.h"

namespace tp {

// Upper bound of the workspace one call may use.  Every GPU the library runs
// on holds one copy of the array until the process ends.
constexpr size_t kStaticScratchBytes = 64ull << 20;

static __device__ __align__(256) char scratch[kStaticScratchBytes];

// Device address of `scratch` per device, looked up once per device with that
// device current.  (In host code the array's name is a host-side stand-in and
// must never be passed to a kernel.)
constexpr int kMaxDevices = 64;
static void *g_scratch_dev[kMaxDevices] = {};
static std::mutex g_scratch_mu;

static tp_status scratch_address(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(TP_E_UNSUPPORTED, "device index beyond the static scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(TP_E_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_dev[dev] = ptr;
    }
    *out = g_scratch_dev[dev];
    return TP_OK;
}

static size_t al256(size_t n) { return (n + 255) & ~(size_t)255; }

// Workspace of one application to nrhs columns, as toeplitz_matvec uses it in
// the plan: two transform grids [max(Ny Px, Px Py)][bc nrhs] (complex128
// slots; bc channels per cell), the rim slab partials [nslab][Nr][nrhs], and
// for a half spectrum the mirror parts [bc / 8][Ny][Px - kxh][bc], and the
// queue and counters of the persistent multi-column launch (256 bytes).
struct StaticLayout {
    size_t grid, rimpart, ypart, total;
};
static StaticLayout static_layout(tp_plan p, int nrhs) {
    StaticLayout L;
    const size_t gpts = std::max((size_t)p->Ny * p->Px, (size_t)p->Px * p->Py);
    L.grid = al256(gpts * (size_t)p->bc * nrhs * 16);
    L.rimpart = al256((size_t)p->rim_nslab * (p->Nr ? p->Nr : 1) * nrhs * 16);
    L.ypart = p->half ? al256((size_t)((p->bc + 7) / 8) * p->Ny * (p->Px - p->kxh) * p->bc * 16) : 0;
    L.total = 2 * L.grid + L.rimpart + L.ypart + 256;    // + the persistent launch's counters
    return L;
}

}  // namespace tp

using namespace tp;

extern "C" {

size_t toeplitz_static_scratch_bytes(void) { return kStaticScratchBytes; }

tp_status toeplitz_matvec_static(tp_plan p, tp_prec which, const void *x, long ldx, void *y, long ldy, int nrhs,
                                 void *hip_stream) {
    tp_status s = check_apply(p, which, x, ldx, y, ldy, nrhs);
    if (s != TP_OK) return s;
    const StaticLayout L = static_layout(p, nrhs);
    if (L.total > kStaticScratchBytes)
        return fail(TP_E_INVAL, "this application needs " + std::to_string(L.total) +
                                    " bytes of workspace; the static scratch holds " +
                                    std::to_string(kStaticScratchBytes));
    void *base = nullptr;
    if ((s = scratch_address(&base)) != TP_OK) return s;
    // a copy of the plan record that points the workspace at the scratch
    tp_plan_s q = *p;
    char *b = static_cast<char *>(base);
    q.gridA = b;
    q.gridB = b + L.grid;
    q.rim_part = b + 2 * L.grid;
    q.ypart = L.ypart ? b + 2 * L.grid + L.rimpart : nullptr;
    q.fctr = reinterpret_cast<int *>(b + 2 * L.grid + L.rimpart + L.ypart);
    hipStream_t st = (hipStream_t)hip_stream;
    hipError_t e;
    if (which == TP_FP64)
        e = matvec_fp64(&q, Cols<const c128>{(const c128 *)x, ldx, nullptr}, Cols<c128>{(c128 *)y, ldy, nullptr},
                        nrhs, st);
    else if (which == TP_FP32)
        e = matvec_fp32(&q, Cols<const c64>{(const c64 *)x, ldx, nullptr}, Cols<c64>{(c64 *)y, ldy, nullptr}, nrhs,
                        st);
    else
        e = matvec_fp32_wide(&q, Cols<const c128>{(const c128 *)x, ldx, nullptr}, Cols<c128>{(c128 *)y, ldy, nullptr},
                             nrhs, st);
    if (e != hipSuccess) return hip_fail(e, "matvec launch");
    return TP_OK;
}

}  // extern "C"
