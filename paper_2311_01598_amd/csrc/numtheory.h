// numtheory.h -- host number theory of the plans: primality, the default
// moduli, the smallest primitive 2N-th root of unity, and modular helpers,
// for 30-bit towers in 32-bit words and ~60-bit towers in 64-bit words.
// Plain C++ (no HIP): the same file builds into the library and, for the
// sanitizer test, into a host program on its own.
#pragma once
#include <cstdint>

namespace ks {

// ---- 32-bit words
uint32_t pow_mod(uint64_t b, uint64_t e, uint32_t q);
// Deterministic Miller-Rabin, bases {2, 7, 61}: exact below 4,759,123,141.
bool is_prime_u64(uint64_t n);
// Primes 2^30 - t 2N + 1 (t = 1, 2, ...) above 2^29: the first `count`.
int ntt_primes(uint32_t log_n, uint32_t count, uint32_t *out);
// The smallest x with x^N = -1 (mod q), or 0 if q is not a prime = 1 mod 2N.
uint32_t min_root_2n(uint32_t q, uint32_t log_n);

// ---- 64-bit words
uint64_t mulmod64(uint64_t a, uint64_t b, uint64_t q);
uint64_t powmod64(uint64_t b, uint64_t e, uint64_t q);
uint64_t invmod64(uint64_t a, uint64_t q);  // q prime
uint64_t shoup64(uint64_t w, uint64_t q);   // floor(w 2^64 / q), w < q
uint64_t mont64(uint64_t w, uint64_t q);    // (w mod q) 2^64 mod q
// Deterministic Miller-Rabin, the first twelve primes as bases: exact for
// every 64-bit n.
bool is_prime64(uint64_t n);
// Primes 2^60 - t 2N + 1 (t = 1, 2, ...) above 2^59: the first `count`.
int ntt_primes64(uint32_t log_n, uint32_t count, uint64_t *out);
// The smallest x with x^N = -1 (mod q), or 0 if q is not a prime = 1 mod 2N.
uint64_t min_root64(uint64_t q, uint32_t log_n);

}  // namespace ks
