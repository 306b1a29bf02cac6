// probe.hip -- the 30-bit modular arithmetic of the kernels, applied
// element-wise to caller arrays so that a test can compare every primitive
// with a*b mod q directly (not part of the method).
#include <hip/hip_runtime.h>

#include "ks.h"
#include "modarith.h"

namespace ks {
namespace {

constexpr uint32_t kProbeOut = 8;

// Element i: a = a[i], b = b[i] (any 32-bit words), w = w[i] mod q.  Each
// primitive gets its operands reduced into the range it is specified for.
__global__ __launch_bounds__(256) void k_arith_probe(ModQ m, double qrecip, uint32_t n, const uint32_t *a,
                                                     const uint32_t *b, const uint32_t *w, uint32_t *out) {
  const uint32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const uint32_t q = m.q, ai = a[i], bi = b[i], wc = w[i] % q;
  const uint32_t wp = shoup_companion(wc, q, qrecip);  // as the OC tiles derive it
  uint32_t *o = out + (size_t)i * kProbeOut;
  o[0] = csub(mul_shoup(ai, wc, wp, q), q);  // a w mod q
  o[1] = redc64(mad64(ai % q, bi % q, 0), m);  // a b 2^-32 mod q
  uint64_t s = 0;  // sum of the 16 products from element i on (cyclically), 2^-32
  for (uint32_t k = 0; k < 16; k++) {
    const uint32_t j = (i + k) % n;
    s = mad64(a[j] % q, b[j] % q, s);
  }
  o[2] = redc64(s, m);
  uint32_t x = ai % (4 * q), y = bi % (4 * q);
  bfly_ct(x, y, 0u - wc, wp, q);  // (x + w y, x - w y), [0, 4q)
  o[3] = x;
  o[4] = y;
  uint32_t u = ai % (2 * q), v = bi % (2 * q);
  bfly_gs(u, v, wc, wp, q);  // (u + v, (u - v) w), [0, 2q)
  o[5] = u;
  o[6] = v;
  o[7] = canon4(ai % (4 * q), q);
}

}  // namespace
}  // namespace ks

extern "C" ks_status_t ks_arith_probe(uint32_t q, uint32_t n, const uint32_t *a, const uint32_t *b,
                                      const uint32_t *w, uint32_t *out, void *stream) {
  if (!a || !b || !w || !out || n == 0) return KS_ERR_INVALID_ARG;
  if (!(q & 1u) || q <= (1u << 29) || q >= (1u << 30)) return KS_ERR_INVALID_ARG;
  uint32_t inv = 1;  // q^-1 mod 2^32 by Newton's iteration
  for (int k = 0; k < 5; k++) inv *= 2u - q * inv;
  const ks::ModQ m{q, 0u - inv, (uint32_t)((1ull << 32) / q), 0};
  hipLaunchKernelGGL(ks::k_arith_probe, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, m,
                     4294967296.0 / (double)q, n, a, b, w, out);
  return hipGetLastError() == hipSuccess ? KS_OK : KS_ERR_DEVICE;
}
