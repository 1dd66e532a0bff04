// mfc_rhs_noalloc: the right-hand side of mfc_rhs on the split kernels, for
// callers that cannot allocate device memory.  Its one scratch buffer, the
// x+y part of every cell (nvar arrays of the padded grid, in the storage
// type), lives in a file-scope device array of fixed size that every GPU the
// library runs on holds until the process ends; nothing is allocated per
// call.  The kernels are those of mfc_rhs with MFC_KERNEL_SPLIT.
#include <mutex>

#include "internal.h"

namespace mfc {
namespace {

// 64 MiB: the x+y part of a grid of up to 1,198,372 padded cells in FP64
// (about 100^3 interior cells) or 2,396,745 in FP32 storage.
constexpr size_t kScratchBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` on each device, taken once per device with that
// device current (each device holds its own copy of the array).  In host code
// the array's name is not a device address: only these pointers are passed
// to the kernels.
constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void *g_scratch[kMaxDevices];

int scratch_address(int device, void **out)
{
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_scratch[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_status(e, "address of the scratch array");
        if (!p) return fail(MFC_E_HIP, "address of the scratch array is null");
        g_scratch[device] = p;
    }
    *out = g_scratch[device];
    return MFC_OK;
}

}  // namespace
}  // namespace mfc

extern "C" int mfc_rhs_noalloc(const mfc_grid_desc *desc, const void *q, void *rhs, int *flag_dev, void *stream)
{
    using namespace mfc;
    if (!desc || !q || !rhs || !flag_dev) return fail(MFC_E_ARG, "null argument");
    if (q == rhs) return fail(MFC_E_ARG, "q and rhs must be distinct");
    int st = validate_desc(desc);
    if (st != MFC_OK) return st;
    if (desc->ndim != 3) return fail(MFC_E_UNSUPPORTED, "mfc_rhs_noalloc is 3D only (the split kernels)");
    if (desc->recon == MFC_RECON_LEARNED) return fail(MFC_E_UNSUPPORTED, "mfc_rhs_noalloc: no learned routing");
    for (int d = 0; d < 3; d++) {
        if (desc->faces[d]) return fail(MFC_E_UNSUPPORTED, "mfc_rhs_noalloc: uniform cells only");
        if (desc->bc[2 * d] == MFC_BC_CHARACTERISTIC || desc->bc[2 * d + 1] == MFC_BC_CHARACTERISTIC)
            return fail(MFC_E_UNSUPPORTED, "mfc_rhs_noalloc: no characteristic boundaries");
    }
    Grid g;
    make_grid(*desc, g);
    const bool fp32 = desc->precision == MFC_FP32_MIXED;
    const uint64_t need = (uint64_t)(4 + g.ndim) * (uint64_t)g.vstride * (fp32 ? 4u : 8u);
    if (need > kScratchBytes)
        return fail(MFC_E_ARG, "mfc_rhs_noalloc: grid too large for its 64 MiB scratch (nvar x padded cells x element "
                               "size must not exceed 67108864 bytes)");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_status(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(MFC_E_UNSUPPORTED, "device index beyond 63");
    void *lxy = nullptr;
    if ((st = scratch_address(dev, &lxy)) != MFC_OK) return st;
    return launch_rhs_split_raw(g, fp32, q, rhs, lxy, flag_dev, (hipStream_t)stream);
}
