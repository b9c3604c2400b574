// run_paths without device allocations: the workspace is a fixed device array of this library
// (one per GPU, held until the process ends), for callers that cannot allocate device memory.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "sf_host.hpp"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

// The workspace of run_paths_noalloc.  In host code its name stands for a host-side symbol, not
// a device address: host code uses only the per-device address from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};

}  // namespace

extern "C" int run_paths_noalloc(sf_circuit_t *c, const uint64_t *path_ids, uint64_t path_begin, uint64_t n_paths,
                                 const uint64_t *bitstrings, size_t n_bits, double *amps, uint32_t flags,
                                 void *hip_stream)
{
    const uint32_t dev_io = SF_OUT_ON_DEVICE | SF_BITS_ON_DEVICE;
    if ((flags & dev_io) != dev_io)
        return sf::set_error(SF_ERR_INVALID, "run_paths_noalloc: bitstrings and amplitudes must be device "
                                             "buffers (SF_BITS_ON_DEVICE | SF_OUT_ON_DEVICE)");
    if (flags & SF_TIMING) return sf::set_error(SF_ERR_INVALID, "run_paths_noalloc: SF_TIMING is not accepted");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return sf::set_error(SF_ERR_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return sf::set_error(SF_ERR_UNSUPPORTED, "device index beyond 63");
    void *ws = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_scratch[dev]) {
            void *p = nullptr;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p)
                return sf::set_error(SF_ERR_DEVICE, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
            g_scratch[dev] = p;
        }
        ws = g_scratch[dev];
    }
    const int rc = sf::run_paths_in(c, path_ids, path_begin, n_paths, bitstrings, n_bits, amps, flags, hip_stream, ws,
                                    kScratchBytes);
    if (rc == SF_ERR_OOM)
        return sf::set_error(SF_ERR_OOM, std::string("run_paths_noalloc: the request needs more than the library's "
                                                     "64 MiB workspace (") + last_error() + ")");
    return rc;
}
