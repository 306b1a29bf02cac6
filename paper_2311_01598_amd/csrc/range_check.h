// range_check.h -- the range-check build's assertions on the lazy ranges.
//
// The arithmetic keeps intermediate words in lazy ranges ([0, 4q) and
// [0, 2q) for the 30-bit butterflies, [0, 8q) and [0, 4q) for the 64-bit
// ones) and sums products in 64-bit accumulators without reducing each
// term.  Those bounds are what make the results exact, so a build compiled
// with KS_CHECK_RANGES (libks_check.so) tests each one where the arithmetic
// relies on it.  A violated bound adds one to a counter in device memory
// (an ordinary vector atomic) and records its code; the computation goes
// on, no kernel traps.  ks_range_violations (include/ks.h) reads and
// clears the counters.  In the normal build (libks.so) KS_RANGE compiles to
// nothing.
//
// Without relocatable device code every compile unit holds its own device
// variables, so each HIP unit that includes this header has its own counter
// and registers a reader for it when the library loads (host-only units
// include it through the plan header and hold no counter).
#pragma once
#include <stdint.h>

// Codes of the checked bounds (the code of one violation is reported).
enum KsRangeCode : uint32_t {
  KS_RC_CT_IN = 1,       // 30-bit Cooley-Tukey butterfly input >= 4q
  KS_RC_GS_IN = 2,       // 30-bit Gentleman-Sande butterfly input >= 2q
  KS_RC_SHOUP_OUT = 3,   // 30-bit Shoup product >= 2q
  KS_RC_MAC_OPND = 4,    // 30-bit multiply-accumulate operand >= 2^30
  KS_RC_MAC_WRAP = 5,    // 64-bit accumulator wrapped
  KS_RC_REDC_OUT = 6,    // 30-bit REDC result not canonical (or, strict, >= q/2)
  KS_RC_CANON4_IN = 7,   // [0, 4q) -> [0, q) input >= 4q
  KS_RC64_CT_IN = 11,    // 64-bit Cooley-Tukey butterfly input >= 8q
  KS_RC64_GS_IN = 12,    // 64-bit Gentleman-Sande butterfly input >= 4q
  KS_RC64_SHOUP4 = 13,   // 64-bit estimated-quotient Shoup product >= 4q
  KS_RC64_SHOUP = 14,    // 64-bit Shoup product >= 2q
  KS_RC64_MAC_OPND = 15, // 64-bit multiply-accumulate half >= 2^30
  KS_RC64_MAC_WRAP = 16, // a partial sum of the 64-bit accumulator wrapped
  KS_RC64_REDC_IN = 17,  // 64-bit REDC input >= m 2^64
  KS_RC64_FWD_IN = 18,   // forward transform's last word >= 8q
};

#ifdef KS_CHECK_RANGES
namespace ks_range {
typedef int (*reader_t)(uint32_t *count, uint32_t *code, int reset);
typedef int (*strict_t)(int on);
// Defined once in the library (api.cpp): the registry of the units' readers.
void register_unit(reader_t read, strict_t strict);
}  // namespace ks_range
#endif

#if defined(KS_CHECK_RANGES) && defined(__HIP__)
#include <hip/hip_runtime.h>
namespace ks_range {
// This unit's counter: [0] violations, [1] the code of one of them; and its
// strict flag, which makes the REDC check demand results below q/2 so that
// a test can show the counters are live on ordinary inputs.
static __device__ uint32_t g_fail[2];
static __device__ uint32_t g_strict;
__device__ __forceinline__ void note(uint32_t code) {
  atomicAdd(&g_fail[0], 1u);
  atomicCAS(&g_fail[1], 0u, code);
}
__device__ __forceinline__ bool strict() { return *(volatile uint32_t *)&g_strict != 0; }
static int read_unit(uint32_t *count, uint32_t *code, int reset) {
  uint32_t v[2] = {0, 0};
  if (hipMemcpyFromSymbol(v, HIP_SYMBOL(g_fail), sizeof v) != hipSuccess) return -1;
  if (reset) {
    const uint32_t z[2] = {0, 0};
    if (hipMemcpyToSymbol(HIP_SYMBOL(g_fail), z, sizeof z) != hipSuccess) return -1;
  }
  *count += v[0];
  if (v[0] && !*code) *code = v[1];
  return 0;
}
static int set_strict(int on) {
  const uint32_t v = on ? 1u : 0u;
  return hipMemcpyToSymbol(HIP_SYMBOL(g_strict), &v, sizeof v) == hipSuccess ? 0 : -1;
}
static const int g_registered = (register_unit(read_unit, set_strict), 0);
}  // namespace ks_range
#define KS_RANGE(cond, code)             \
  do {                                   \
    if (!(cond)) ::ks_range::note(code); \
  } while (0)
#define KS_RANGE_STRICT() (::ks_range::strict())
#else
#define KS_RANGE(cond, code) \
  do {                       \
  } while (0)
#define KS_RANGE_STRICT() false
#endif
