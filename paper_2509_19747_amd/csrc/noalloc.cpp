// rr_apply_operator_noalloc: the operator product y = (A + mu I) u of
// rr_apply_operator (the matvec of every Krylov iteration, Section 6) for callers
// that cannot allocate device memory (code under graph capture, tight serving
// loops).  Every buffer the product needs beyond u and y -- the point records of
// a kernel operator, the float32 copy of a dense A, the partial-sum slots and the
// dot partials -- is carved from one file-scope device array, `scratch`.
//
// The array's host-side name is not a device address: its address on each device
// is taken once per device with hipGetSymbolAddress (first call on that device,
// with the device current) and only that pointer is handed to kernels.  Calls on
// one device share the array and it keeps the last call's contents; calls that
// overlap on one device race.  Nothing here allocates, frees or synchronises.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "ctx.hpp"

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;   // 64 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device.
void* scratch_on_device() {
    int dev = 0;
    RR_HIP(hipGetDevice(&dev));
    RR_REQUIRE(dev >= 0 && dev < kMaxDevices, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            throw rr::RrError{RR_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
        }
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

// Bump layout inside the scratch array (256-byte aligned pieces).
struct Carve {
    size_t off = 0;
    size_t take(size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) / 256 * 256;
        return o;
    }
};

struct Layout {
    size_t sqn = 0, xa = 0, xd = 0, hd = 0, a32 = 0, part = 0, ws = 0, total = 0;
};

Layout layout_for(const rr_operator& A, int32_t prec) {
    Layout L;
    Carve c;
    const int64_t n = A.n;
    if (rr::is_kernel(A)) {
        const int dm = rr::kernel_record_len(A.d);
        L.sqn = c.take((size_t)n * sizeof(float));
        L.xa = c.take((size_t)n * dm * sizeof(float));
        L.xd = c.take((size_t)n * dm * sizeof(double));
        L.hd = c.take((size_t)n * sizeof(double));
        L.part = c.take((size_t)rr::kernel_matvec_blocks(n) * sizeof(double));
        L.ws = c.take((rr::kernel_matvec_ws_doubles_for(n, A.d, 1, prec == RR_PREC_FP64) + 1) * sizeof(double));
    } else {
        if (prec != RR_PREC_FP64) L.a32 = c.take((size_t)n * n * sizeof(float));
        L.part = c.take((size_t)rr::dense_matvec_blocks(n) * sizeof(double));
    }
    L.total = c.off;
    return L;
}

}  // namespace

using namespace rr;

extern "C" rr_status rr_apply_operator_noalloc(const rr_operator* A, double mu, int32_t prec, const double* u,
                                               double* y, void* hip_stream) {
    return guarded([&]() -> rr_status {
        validate_operator(A);
        RR_REQUIRE(u != nullptr && y != nullptr, "u or y is null");
        RR_REQUIRE(std::isfinite(mu), "mu must be finite");
        RR_REQUIRE(prec >= 0 && prec <= 2, "unknown precision");
        const Layout L = layout_for(*A, prec);
        if (L.total > kScratchBytes)
            throw RrError{RR_EINVAL, "operator too large for the no-allocation scratch: needs " +
                                         std::to_string(L.total) + " bytes, the scratch holds " +
                                         std::to_string(kScratchBytes)};
        require_device();
        unsigned char* base = (unsigned char*)scratch_on_device();
        hipStream_t st = (hipStream_t)hip_stream;
        const int64_t n = A->n;
        double* part = (double*)(base + L.part);
        if (is_kernel(*A)) {
            KernelOp k;
            k.kind = A->kind;
            k.n = n;
            k.d = A->d;
            k.pts = A->pts;
            k.dm = kernel_record_len(A->d);
            k.kconst = A->kconst;
            k.scale = A->scale;
            k.sqn = (const float*)(base + L.sqn);
            k.xa = (const float*)(base + L.xa);
            k.xd = (const double*)(base + L.xd);
            k.hd = (const double*)(base + L.hd);
            launch_sqnorms(A->pts, n, A->d, (float*)(base + L.sqn), st);
            launch_point_records(A->pts, n, A->d, k.dm, (float*)(base + L.xa), st);
            launch_point_records64(A->pts, n, A->d, k.dm, kernel_g64(A->kind, A->kconst), (double*)(base + L.xd),
                                   (double*)(base + L.hd), st);
            launch_kernel_matvec(k, prec == RR_PREC_FP64, u, mu, y, part, (double*)(base + L.ws), nullptr, st);
        } else if (prec != RR_PREC_FP64) {
            float* a32 = (float*)(base + L.a32);
            launch_copy_mat(DT_F64, A->A, A->lda, DT_F32, a32, n, n, n, st);
            launch_dense_matvec(DT_F32, n, a32, n, u, mu, y, part, nullptr, st);
        } else {
            launch_dense_matvec(DT_F64, n, A->A, A->lda, u, mu, y, part, nullptr, st);
        }
        RR_HIP(hipGetLastError());
        return RR_OK;
    });
}

extern "C" size_t rr_noalloc_scratch_bytes(void) { return kScratchBytes; }
