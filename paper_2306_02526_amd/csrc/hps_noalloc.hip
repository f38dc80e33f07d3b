// hps_solve_noalloc: the FP64 solve of hps_solve (Algorithm 1 of Sec. 2.1 with the body
// load and interface jumps) for callers that cannot allocate device memory.
//
// hps_solve's kernels write their intermediate data (leaf boundary values, particular
// solutions and fluxes, per-level fluxes, boundary values and w3, split-K partials and
// arrival counters) into a workspace that hps_build allocated with the operator.  This
// variant runs the same kernels, in the same order, on a workspace carved out of one
// file-scope device array instead, so it performs no allocation of any kind: usable under
// HIP graph capture, in serving loops and wherever hipMalloc is not allowed.
//
// The array is per device (every GPU the library runs on holds its own copy until the
// process ends).  Host code never passes the array's name to a kernel: its device address
// is looked up once per device with hipGetSymbolAddress, and the kernels receive that
// address through their argument records.  All calls on one GPU share the array, so
// calls that overlap on one GPU (two streams, two threads) race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "hps_internal.h"

using namespace hps;

namespace {
constexpr int64_t kScratchBytes = HPS_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

// Device address of this device's copy of `scratch` (looked up on the first call per device).
static int scratch_address(void **out) {
    int dev = -1;
    HPS_HIP(hipGetDevice(&dev));
    CHECK_ARG(dev >= 0 && dev < kMaxDevices, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            hps_set_error("hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
            return HPS_EDEVICE;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return HPS_OK;
}

extern "C" int hps_solve_noalloc(hps_op *op, int nrhs, const double *body, const double *dirichlet,
                                 const double *jump, double *u, void *stream) {
    CHECK_ARG(op != nullptr, "op is NULL");
    CHECK_ARG(op->ncomp == 1 && !(op->flags & HPS_FP32_IR),
              "hps_solve_noalloc takes real operators built with HPS_FP64");
    CHECK_ARG(nrhs >= 0, "nrhs must be >= 0");
    if (nrhs == 0) return HPS_OK;
    CHECK_ARG(body != nullptr && u != nullptr, "body and u are required");
    TRY(check_device_ptr(body, "body"));
    TRY(check_device_ptr(dirichlet, "dirichlet"));
    TRY(check_device_ptr(jump, "jump"));
    TRY(check_device_ptr(u, "u"));
    int64_t cnt_off = 0, cnt_bytes = 0;
    thread_local Workspace ws;   // host-side record of the carve-up (its level list grows once)
    const int64_t need = workspace_layout(op, nullptr, &ws, &cnt_off, &cnt_bytes);
    if (need > kScratchBytes) {
        hps_set_error("hps_solve_noalloc: this operator's solve needs %lld bytes of scratch, the maximum is %lld",
                      (long long)need, (long long)kScratchBytes);
        return HPS_EINVAL;
    }
    void *base = nullptr;
    TRY(scratch_address(&base));
    workspace_layout(op, static_cast<char *>(base), &ws, &cnt_off, &cnt_bytes);
    hipStream_t st = (hipStream_t)stream;
    // the array keeps the previous call's contents: the split-K arrival counters must
    // start at zero (a fill kernel, so that the call can be captured into a graph)
    if (cnt_bytes) TRY(launch_zero(reinterpret_cast<double *>(static_cast<char *>(base) + cnt_off), cnt_bytes / 8, st));
    for (int r = 0; r < nrhs; ++r) {
        LeafPhase upp;
        upp.up = LU_BODY;
        upp.body = body + (int64_t)r * op->n_int;
        TRY(launch_leaf(op, false, upp, st, &ws));
        TRY(launch_levels(op, false, (jump && op->n_iface) ? jump + (int64_t)r * op->n_iface : nullptr,
                          dirichlet ? dirichlet + (int64_t)r * op->n_bdry : nullptr, st, &ws));
        LeafPhase dn;
        dn.down = LD_WRITE_U;
        dn.u_out = u + (int64_t)r * op->N;
        TRY(launch_leaf(op, false, dn, st, &ws));
    }
    return HPS_OK;
}
