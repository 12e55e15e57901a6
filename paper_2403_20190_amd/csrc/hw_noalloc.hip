// hw_noalloc.hip -- homomorphic training (Alg. 6) for callers that cannot
// allocate device memory.  The training workspace and the device copy of the
// permutation live in `scratch`, a fixed device array of this file: each GPU
// the library runs on holds its own copy from the first call on that GPU
// until the process ends.  The calls on one GPU share that copy, so calls
// whose work overlaps on one GPU (different streams, threads or contexts)
// race; the caller serialises them.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "../../include/hwisard.h"
#include "hw_ctx.h"

static __device__ __align__(256) uint32_t scratch[HW_NOALLOC_SCRATCH_BYTES / 4];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
uint32_t* g_ptr[MAX_DEVICES] = {};  // device address of `scratch` on each GPU, once resolved

// The device address of `scratch` on `device`, which must be current.  In host
// code the array's name only stands in for the symbol; the address a kernel
// may use is the one hipGetSymbolAddress returns for the current device.
hw_status scratch_on(int device, uint32_t** out) {
  if (device < 0 || device >= MAX_DEVICES) return fail(HW_EINVAL, "device %d out of range", device);
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_ptr[device]) {
    uint32_t* p = nullptr;
    HIP_TRY(hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(HW_EDEVICE, "no device address for the scratch array on device %d", device);
    g_ptr[device] = p;
  }
  *out = g_ptr[device];
  return HW_OK;
}

}  // namespace

extern "C" hw_status hw_wisard_train_encrypted_noalloc(hw_ctx* c, const hw_wisard_shape* sh, const uint32_t* x_rgsw,
                                                       const uint32_t* y_rgsw, uint64_t n, uint32_t* model,
                                                       uint32_t* class_count, hipStream_t st) {
  CHECK(enter(c));
  Dims d;
  CHECK(check_shape(c, sh, &d));
  if (n == 0) return ok();
  if (!x_rgsw || !model) return fail(HW_EINVAL, "null buffer");
  if (d.L > 0 && !y_rgsw) return fail(HW_EINVAL, "null label ciphertexts");
  // scratch = [permutation, padded to 256 bytes][per-sample training workspace x n_sub]
  const size_t perm_bytes = ((size_t)sh->s * 4 + 255) / 256 * 256;
  const size_t per_sample = train_ws_per_sample(c, d);
  if (perm_bytes + per_sample > (size_t)HW_NOALLOC_SCRATCH_BYTES)
    return fail(HW_EINVAL,
                "this shape needs %zu bytes of workspace per sample plus %zu for the permutation; the "
                "no-allocation scratch holds %llu bytes (use hw_wisard_train_encrypted)",
                per_sample, perm_bytes, (unsigned long long)HW_NOALLOC_SCRATCH_BYTES);
  uint32_t* base = nullptr;
  CHECK(scratch_on(c->device, &base));
  // the permutation is written by a kernel (nothing is staged on the host)
  HIP_TRY(hw::launch_perm(sh->s, sh->perm_seed, base, st));
  CHECK(train_core(c, sh, d, base, x_rgsw, y_rgsw, n, model, class_count, base + perm_bytes / 4,
                   (size_t)HW_NOALLOC_SCRATCH_BYTES - perm_bytes, st, false, false));
  return ok();
}
