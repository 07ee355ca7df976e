// read_noalloc.hip -- lbm_read_fields_noalloc: the read-back of
// lbm_read_fields through a fixed device staging array of this library
// instead of a device allocation per call.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/lbm.h"
#include "handle.hpp"
#include "lattice_host.hpp"
#include "pflbm.hpp"

using namespace pflbm;

// Staging of lbm_read_fields_noalloc.  Every GPU the library runs on holds
// its own copy from module load until the process ends; host code reaches it
// only through the device address hipGetSymbolAddress returns on that GPU.
static __device__ __align__(256) double scratch[LBM_NOALLOC_MAX_DOUBLES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of the scratch array on device dev, looked up once per
// device with that device current.
int scratch_address(int dev, double** out) {
    if (dev < 0 || dev >= MAX_DEVICES) {
        set_error("device %d outside [0, %d)", dev, MAX_DEVICES);
        return LBM_E_INVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
            return LBM_E_DEVICE;
        }
        g_scratch_ptr[dev] = (double*)p;
    }
    *out = g_scratch_ptr[dev];
    return LBM_OK;
}

}  // namespace

extern "C" int lbm_read_fields_noalloc(lbm_handle* h, uint32_t mask, double* phi, double* P,
                                       double* u, double* pops) {
    if (!h) { set_error("handle is NULL"); return LBM_E_INVAL; }
    const size_t nd = read_staging_elems(h->hdesc, mask, phi, P, u, pops);
    if (nd > (size_t)LBM_NOALLOC_MAX_DOUBLES) {
        set_error("read-back of %zu doubles exceeds the fixed staging of %u doubles", nd,
                  (unsigned)LBM_NOALLOC_MAX_DOUBLES);
        return LBM_E_INVAL;
    }
    hipError_t e = hipSetDevice(h->device);
    if (e != hipSuccess) { set_error("hipSetDevice(%d): %s", h->device, hipGetErrorString(e)); return LBM_E_DEVICE; }
    double* buf = nullptr;
    const int rc = scratch_address(h->device, &buf);
    if (rc != LBM_OK) return rc;
    e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) { set_error("hipStreamSynchronize: %s", hipGetErrorString(e)); return LBM_E_DEVICE; }
    return read_lattice_staged(h->p.storage, h->hdesc, (int)(h->step & 1), h->ddesc, h->dtiles,
                               h->ntiles, h->dwalls, h->nwalls, mask, phi, P, u, pops, buf, h->stream);
}
