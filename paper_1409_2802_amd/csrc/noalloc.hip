// Interpolative decompositions without device allocation: the QR exchange
// slots and the solve's scratch come from a file-scope device array, which
// each GPU holds once for the life of the process.
#include <mutex>

#include "ffc_internal.h"

namespace ffc {
namespace {

// In host code `scratch` only names the symbol; its device address on the
// current GPU comes from hipGetSymbolAddress (kept per device below).
__device__ __align__(256) unsigned char scratch[FFC_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[64] = {};

// This device's copy of `scratch`, looked up once per device.
ffc_status scratch_on_current_device(unsigned char*& out) {
  int dev = 0;
  FFC_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) {
    set_error("device index above 63");
    return FFC_ERR_INVALID_ARG;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    unsigned char* p = nullptr;
    FFC_HIP_TRY(hipGetSymbolAddress(reinterpret_cast<void**>(&p), HIP_SYMBOL(scratch)));
    if (!p) {
      set_error("hipGetSymbolAddress returned no address for the scratch array");
      return FFC_ERR_HIP;
    }
    g_scratch_ptr[dev] = p;
  }
  out = g_scratch_ptr[dev];
  return FFC_OK;
}

ffc_status fail(ffc_status code, const char* msg) {
  set_error(msg);
  return code;
}

}  // namespace
}  // namespace ffc

using namespace ffc;

extern "C" ffc_status ffc_interp_decomp_noalloc(double* A_dev, int32_t batch, int32_t s, int32_t n, double tol,
                                                int32_t max_rank, int32_t* rank_dev, int32_t* piv_dev, double* P_dev,
                                                void* stream) {
  if (batch < 0) return fail(FFC_ERR_INVALID_ARG, "batch must be >= 0");
  if (s < 1 || n < 1) return fail(FFC_ERR_INVALID_ARG, "s and n must be >= 1");
  if (s > 1024) return fail(FFC_ERR_INVALID_ARG, "s above 1024 needs the streamed QR, which allocates");
  if (max_rank < 1) return fail(FFC_ERR_INVALID_ARG, "max_rank must be >= 1");
  if (!(tol >= 0.0)) return fail(FFC_ERR_INVALID_ARG, "tol must be >= 0");
  if (batch == 0) return FFC_OK;
  if (!A_dev || !rank_dev || !piv_dev || !P_dev) return fail(FFC_ERR_INVALID_ARG, "NULL pointer");
  if (!device_flag()) return fail(FFC_ERR_HIP, "no device flag");
  unsigned char* sp = nullptr;
  FFC_TRY(scratch_on_current_device(sp));
  IdBatch bt{};
  bt.A = A_dev;
  bt.a_stride = (int64_t)s * n;
  bt.lda = s;
  bt.s_uniform = s;
  bt.n_uniform = n;
  bt.s_max = s;
  bt.n_max = n;
  bt.tol = tol;
  bt.max_rank = max_rank;
  bt.rank = rank_dev;
  bt.piv = piv_dev;
  bt.piv_stride = n;
  bt.P = P_dev;
  bt.p_stride = (int64_t)max_rank * n;
  bt.p_ld = n;
  return launch_interp_decomp_fixed(bt, batch, sp, FFC_NOALLOC_SCRATCH_BYTES, (hipStream_t)stream);
}
