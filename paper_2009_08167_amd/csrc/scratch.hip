// Fixed device scratch for the entry points that allocate nothing
// (riga_project_noalloc): a file-scope array in the library's code object,
// one copy per GPU, held until the process ends.  Host code never passes the
// array's name to a kernel: its device address is looked up once per device
// (hipGetSymbolAddress, with that device current) and that address is used
// wherever host code needs the memory.
#include <hip/hip_runtime.h>

#include <mutex>

#include "problem.h"

static __device__ __align__(256) double scratch[riga::NOALLOC_SCRATCH_DOUBLES];

namespace riga {
namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[MAX_DEVICES] = {};

}  // namespace

double* noalloc_scratch() {
  int dev = 0;
  HIPCHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) throw Error(RIGA_EUNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw Error(RIGA_EDEVICE, "hipGetSymbolAddress returned a null scratch address");
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  return g_scratch_ptr[dev];
}

}  // namespace riga
