// Operator application that allocates nothing (eigcg_apply_noalloc): for
// callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc).  Its staging fields
// live in a fixed device array of this file instead of the context's
// workspace, which eigcg_apply allocates on first use.
//
// The array is one per GPU the library runs on, held until the process ends.
// Host code never passes the array's name to a kernel or a copy (on the host
// it is only a stand-in symbol): the device address is looked up once per
// device with hipGetSymbolAddress and kept.  Every call on a GPU shares that
// GPU's array, so calls that overlap on one GPU race.
#include <mutex>

#include "engine.h"

namespace eigcg {

constexpr size_t kScratchBytes = (size_t)64 << 20;  // two FP64 fields of up to 16^3 x 32 sites

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// The device address of this GPU's scratch array (looked up on the first
// call on the device, with the device current, and registered with the
// bounds layer so launches into it are checked like the library's own
// allocations).
void* scratch_ptr(int dev) {
  if (dev < 0 || dev >= kMaxDevices) throw ApiError{EIGCG_EINVAL, "device index out of range"};
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) throw HipError{e != hipSuccess ? e : hipErrorInvalidSymbol,
                                              "hipGetSymbolAddress(scratch)"};
    register_span(p, kScratchBytes);
    g_ptr[dev] = p;
  }
  return g_ptr[dev];
}

}  // namespace

size_t noalloc_scratch_bytes() { return kScratchBytes; }

// out = op(in) (M, M^H or A = M^H M in FP64) one column at a time through two
// staging fields in the scratch array: in -> f0 (internal layout); M: f0 -> f1;
// A: then M^H: f1 -> f0.  Every site a kernel reads is written earlier in the
// same call (stencil loads are limited to the lattice sites, not the plane
// padding), so nothing in the array needs clearing between calls.
void apply_op_noalloc(Ctx& c, int op, int nrhs, const void* in_aos, void* out_aos) {
  if (op < EIGCG_OP_M || op > EIGCG_OP_A)
    throw ApiError{EIGCG_EINVAL, "eigcg_apply_noalloc: op must be M, M^H or A (FP64)"};
  const size_t field = c.cs * 16;
  if (2 * field > kScratchBytes)
    throw ApiError{EIGCG_EINVAL, "eigcg_apply_noalloc: two FP64 fields of this lattice need " +
                                     std::to_string(2 * field) + " bytes, the static scratch holds " +
                                     std::to_string(kScratchBytes)};
  int dev = 0;
  c.check(hipGetDevice(&dev), "hipGetDevice");
  if (dev != c.device) throw ApiError{EIGCG_EINVAL, "eigcg_apply_noalloc: the context's device is not current"};
  char* base = static_cast<char*>(scratch_ptr(dev));
  void* f0 = base;
  void* f1 = base + field;
  for (int j = 0; j < nrhs; ++j) {
    const double2* src = (const double2*)in_aos + (size_t)j * 12 * c.g.V;
    double2* dst = (double2*)out_aos + (size_t)j * 12 * c.g.V;
    c.check(launch_spinor_to_soa(src, f0, kF64, &c.g, 1, c.cs, c.stream), "to soa");
    void* res = f1;
    if (op == EIGCG_OP_A) {
      stencil_store(c, kF64, kOpM, 1, f0, f1);
      stencil_store(c, kF64, kOpMdag, 1, f1, f0);
      res = f0;
    } else {
      stencil_store(c, kF64, op == EIGCG_OP_M ? kOpM : kOpMdag, 1, f0, f1);
    }
    c.check(launch_spinor_from_soa(res, dst, kF64, &c.g, 1, c.cs, c.stream), "from soa");
  }
  c.check(hipStreamSynchronize(c.stream), "sync");
}

}  // namespace eigcg
