// H_eff * psi without any device allocation, for callers that cannot
// allocate (code under HIP graph capture, tight serving loops): its
// intermediates -- T1 = L psi, T2 = the W-mapped T1, the K-contiguous copy of
// psi and the split-K partial products -- live in a file-scope device array
// of fixed size, one copy per GPU, held until the process ends.  In host code
// the array's name is only a host-side stand-in, so its device address is
// looked up once per device at context creation and used everywhere else.
#include <mutex>

#include "d3s_internal.h"

namespace d3s {

constexpr size_t kNoallocScratch = (size_t)64 << 20;   // 64 MiB per GPU

static __device__ __align__(256) unsigned char scratch[kNoallocScratch];

namespace {
constexpr int kMaxDevices = 64;
void* g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }
}  // namespace

size_t noalloc_capacity() { return kNoallocScratch; }

// T1, T2 and the psi copy, each on a 256-byte boundary (the split-K partials
// take whatever is left)
size_t noalloc_bytes(d3s_prec p, int ml, int d, int mr, int wl, int wr) {
  const size_t tsz = (p == D3S_F64) ? 8 : 4;
  const size_t esz = (p == D3S_F64) ? 8 : (p == D3S_F32 ? 4 : 2);
  return up256(tsz * (size_t)ml * wl * d * mr) + up256(esz * (size_t)ml * d * wr * mr) +
         up256(esz * (size_t)ml * d * mr);
}

// with `device` current: the device address of this GPU's copy of the array
void noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) throw Error{D3S_EINVAL, "device index beyond the scratch table"};
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[device]) return;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    throw Error{D3S_EDEVICE, std::string("hipGetSymbolAddress of the scratch array: ") + hipGetErrorString(e)};
  }
  g_scratch[device] = ptr;
}

void op_apply_heff_noalloc(Ctx* c, d3s_prec p, int ml, int d, int mr, int wl, int wr, const void* L,
                           const void* W, const void* R, const void* psi, void* out) {
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    base = (c->device >= 0 && c->device < kMaxDevices) ? g_scratch[c->device] : nullptr;
  }
  if (!base) throw Error{D3S_EDEVICE, "the scratch array of this device was not set up"};
  const size_t need = noalloc_bytes(p, ml, d, mr, wl, wr);
  if (need > kNoallocScratch)
    throw Error{D3S_EINVAL, "apply_heff_noalloc: the product needs " + std::to_string(need) +
                                " bytes of scratch, more than the " + std::to_string(kNoallocScratch) + " available"};
  const size_t tsz = (p == D3S_F64) ? 8 : 4;
  const size_t esz = (p == D3S_F64) ? 8 : (p == D3S_F32 ? 4 : 2);
  char* b = (char*)base;
  void* T1 = b;
  b += up256(tsz * (size_t)ml * wl * d * mr);
  void* T2 = b;
  b += up256(esz * (size_t)ml * d * wr * mr);
  void* psiT = b;
  b += up256(esz * (size_t)ml * d * mr);
  heff_product(c, p, ml, d, mr, wl, wr, L, W, R, psi, out, T1, T2, psiT, b, kNoallocScratch - need, true);
}

}  // namespace d3s
