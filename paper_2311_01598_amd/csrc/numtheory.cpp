// numtheory.cpp -- see numtheory.h.
//
// psi for both word sizes: from a generator c of Z_q^* (the smallest c with
// c^((q-1)/f) != 1 for every prime f | q-1, the factors found by trial
// division), psi_0 = c^((q-1)/2N) is a primitive 2N-th root; the primitive
// 2N-th roots are psi_0^k for odd k, and the smallest of those N values is
// returned.
#include "numtheory.h"

#include <algorithm>
#include <vector>

namespace ks {

namespace {
typedef unsigned __int128 u128;
inline uint64_t mulm(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((u128)a * b % m); }

// Distinct prime factors of m by trial division.
std::vector<uint64_t> prime_factors(uint64_t m) {
  std::vector<uint64_t> f;
  for (uint64_t p = 2; p * p <= m; p += (p == 2 ? 1 : 2))
    if (m % p == 0) {
      f.push_back(p);
      while (m % p == 0) m /= p;
    }
  if (m > 1) f.push_back(m);
  return f;
}

uint64_t smallest_odd_power(uint64_t q, uint64_t psi0, uint64_t n) {
  const uint64_t sq = mulm(psi0, psi0, q);
  uint64_t best = psi0, cur = psi0;
  for (uint64_t k = 1; k < n; k++) {  // psi0^(2k+1)
    cur = mulm(cur, sq, q);
    best = std::min(best, cur);
  }
  return best;
}

uint64_t generator(uint64_t q) {
  const std::vector<uint64_t> f = prime_factors(q - 1);
  for (uint64_t c = 2; c < q; c++) {
    bool ok = true;
    for (uint64_t p : f)
      if (powmod64(c, (q - 1) / p, q) == 1) { ok = false; break; }
    if (ok) return c;
  }
  return 0;
}
}  // namespace

uint32_t pow_mod(uint64_t b, uint64_t e, uint32_t q) { return (uint32_t)powmod64(b, e, q); }

bool is_prime_u64(uint64_t n) {
  if (n < 2) return false;
  for (uint64_t p : {2ull, 3ull, 5ull, 7ull, 11ull, 13ull, 61ull})
    if (n % p == 0) return n == p;
  uint64_t d = n - 1;
  int s = 0;
  while (!(d & 1)) { d >>= 1; s++; }
  for (uint64_t a : {2ull, 7ull, 61ull}) {
    uint64_t x = powmod64(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int i = 1; i < s; i++) {
      x = mulm(x, x, n);
      if (x == n - 1) { comp = false; break; }
    }
    if (comp) return false;
  }
  return true;
}

int ntt_primes(uint32_t log_n, uint32_t count, uint32_t *out) {
  const uint64_t step = 2ull << log_n;
  uint32_t k = 0;
  for (uint64_t c = (1ull << 30) + 1 - step; k < count; c -= step) {
    if (c <= (1ull << 29)) return -1;
    if (is_prime_u64(c)) out[k++] = (uint32_t)c;
  }
  return 0;
}

uint32_t min_root_2n(uint32_t q, uint32_t log_n) {
  const uint64_t two_n = 2ull << log_n;
  if (!is_prime_u64(q) || (q - 1) % two_n) return 0;
  const uint64_t psi0 = powmod64(generator(q), (q - 1) / two_n, q);
  return (uint32_t)smallest_odd_power(q, psi0, two_n / 2);
}

uint64_t mulmod64(uint64_t a, uint64_t b, uint64_t q) { return mulm(a, b, q); }

uint64_t powmod64(uint64_t b, uint64_t e, uint64_t q) {
  uint64_t r = 1 % q;
  b %= q;
  while (e) {
    if (e & 1) r = mulm(r, b, q);
    b = mulm(b, b, q);
    e >>= 1;
  }
  return r;
}

uint64_t invmod64(uint64_t a, uint64_t q) { return powmod64(a, q - 2, q); }
uint64_t shoup64(uint64_t w, uint64_t q) { return (uint64_t)(((u128)w << 64) / q); }
uint64_t mont64(uint64_t w, uint64_t q) { return (uint64_t)(((u128)(w % q) << 64) % q); }

bool is_prime64(uint64_t n) {
  static const uint64_t B[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return false;
  for (uint64_t b : B) {
    if (n == b) return true;
    if (n % b == 0) return false;
  }
  uint64_t d = n - 1;
  int r = 0;
  while (!(d & 1)) { d >>= 1; r++; }
  for (uint64_t b : B) {
    uint64_t x = powmod64(b, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int i = 1; i < r && comp; i++) {
      x = mulm(x, x, n);
      if (x == n - 1) comp = false;
    }
    if (comp) return false;
  }
  return true;
}

int ntt_primes64(uint32_t log_n, uint32_t count, uint64_t *out) {
  const uint64_t two_n = 2ull << log_n;
  uint32_t k = 0;
  for (uint64_t t = 1; k < count; t++) {
    if (t * two_n >= (1ull << 59)) return -1;
    const uint64_t c = (1ull << 60) - t * two_n + 1;
    if (is_prime64(c)) out[k++] = c;
  }
  return 0;
}

uint64_t min_root64(uint64_t q, uint32_t log_n) {
  const uint64_t two_n = 2ull << log_n;
  if (q < 3 || !is_prime64(q) || (q - 1) % two_n) return 0;
  const uint64_t psi0 = powmod64(generator(q), (q - 1) / two_n, q);
  return smallest_odd_power(q, psi0, two_n / 2);
}

}  // namespace ks
