// Factor + selected inversion in a static per-device workspace, for callers
// that cannot allocate device memory (code under HIP graph capture, tight
// serving loops, harnesses that forbid hipMalloc).  The library's own
// file-scope device array serves as the whole workspace of the plan; every
// kernel takes its address, obtained once per device with
// hipGetSymbolAddress.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "kernels.hpp"
#include "plan.hpp"

namespace {
constexpr size_t kStaticBytes = size_t(64) << 20;  // SELINV_STATIC_SCRATCH_BYTES in selinv.h
constexpr int kMaxDevices = 64;
}  // namespace

// The device array: one copy per GPU, held until the process ends.  Host
// code never uses this name as an address (it would be a host-side stand-in);
// it uses the pointer from hipGetSymbolAddress below.
static __device__ __align__(256) unsigned char scratch[kStaticBytes];

namespace {
std::mutex g_mu;
char* g_ptr[kMaxDevices] = {};          // device address of `scratch`, per device
uint64_t g_owner[kMaxDevices] = {};     // plan whose tables the array holds (0: none)
uint64_t g_next_uid = 1;

// the array's device address on the current device (looked up once per device)
hipError_t scratch_ptr(int dev, char** out)
{
    if (!g_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[dev] = (char*)p;
    }
    *out = g_ptr[dev];
    return hipSuccess;
}
}  // namespace

extern "C" selinv_status selinv_factor_invert_static(selinv_plan P, const double* d_valsA, double* d_sel,
                                                     int64_t* bad_col, hipStream_t s)
{
    using namespace selinv;
    if (bad_col) *bad_col = -1;
    if (!P) return set_error(SELINV_EINVAL, "NULL plan");
    if (P->opts.complex_values)
        return set_error(SELINV_EINVAL, "the plan holds complex values (selinv_*_complex)");
    if ((P->nnzA > 0 && !d_valsA) || (P->colptrL.back() > 0 && !d_sel)) return set_error(SELINV_EINVAL, "NULL buffer");
    if (P->lay.total > kStaticBytes)
        return set_error(SELINV_ENOMEM, "the plan's workspace (" + std::to_string(P->lay.total) +
                                            " bytes) exceeds the static scratch of " + std::to_string(kStaticBytes) +
                                            " bytes");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e) return set_error(SELINV_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return set_error(SELINV_EUNSUPPORTED, "device index out of range");
    char* base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        e = scratch_ptr(dev, &base);
        if (e) return set_error(SELINV_EHIP, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
        if (P->static_uid == 0) P->static_uid = g_next_uid++;
        // the tables only when the array holds another plan's
        if (g_owner[dev] != P->static_uid) {
            const hipError_t init = kernels_init();
            if (init) return set_error(SELINV_EHIP, std::string("kernel attributes: ") + hipGetErrorString(init));
            e = upload_tables(P, base, s);
            if (e) {
                g_owner[dev] = 0;
                return set_error(SELINV_EHIP, std::string("table upload: ") + hipGetErrorString(e));
            }
            g_owner[dev] = P->static_uid;
        }
    }
    const DevPtrs D = dev_ptrs_at(P, base, base + P->lay.persist);
    e = factor_levels(P, D, d_valsA, s, nullptr);
    if (!e) e = invert_levels(P, D, d_sel, s, nullptr);
    if (e) return set_error(SELINV_EHIP, std::string("static launch: ") + hipGetErrorString(e));
    if (!bad_col) return SELINV_OK;
    unsigned long long w[2] = {~0ull, 0ull};
    e = hipMemcpyAsync(w, base + P->lay.status, sizeof w, hipMemcpyDeviceToHost, s);
    if (!e) e = hipStreamSynchronize(s);
    if (e) return set_error(SELINV_EHIP, std::string("status read: ") + hipGetErrorString(e));
    if (w[0] != ~0ull) {
        const int64_t col = (int64_t)w[0];
        *bad_col = (col >= 0 && col < P->n) ? P->perm[col] : -1;
        return set_error(SELINV_EPIVOT, "bad pivot at original column " + std::to_string(*bad_col));
    }
    return SELINV_OK;
}
