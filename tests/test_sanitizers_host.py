"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (gcc/g++,
CPU only): the plain-C oracle of both word sizes, driven through key
generation, both key-switch orders, rotations and multiplication at small
N, and the library's host number theory (numtheory.cpp: moduli and roots of
both word sizes), whose outputs must also equal the oracle's.  Any
sanitizer report aborts the program (-fno-sanitize-recover=all)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from oracle import core64 as o64

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]

ORACLE_DRIVER = r"""
#include <stdio.h>
#include <stdlib.h>
#include "ks_oracle.h"
static int run32(uint32_t log_n, uint32_t nq, uint32_t dnum, uint32_t np) {
  oracle_params p = {log_n, nq, dnum, np};
  const uint32_t n = 1u << log_n, el = nq + np;
  uint32_t *m = malloc(sizeof(uint32_t) * el);
  uint32_t *evk = malloc(sizeof(uint32_t) * (size_t)dnum * 2 * el * n);
  uint32_t *d = calloc((size_t)nq * n, sizeof(uint32_t));
  uint32_t *o = malloc(sizeof(uint32_t) * 2 * (size_t)nq * n), *o2 = malloc(sizeof(uint32_t) * 2 * (size_t)nq * n);
  int8_t *s = malloc(n), *s2 = malloc(n);
  if (oracle_moduli(&p, m) || oracle_keygen(&p, m, 5, s, s2, evk) < 0) return 1;
  for (uint32_t i = 0; i < nq; i++) for (uint32_t z = 0; z < n; z++) d[(size_t)i * n + z] = (z * 2654435761u + i) % m[i];
  for (uint32_t lv = 0; lv < nq; lv++) {
    if (oracle_keyswitch(&p, m, lv, evk, d, o) || oracle_keyswitch_oc(&p, m, lv, evk, d, o2)) return 2;
    for (size_t z = 0; z < 2 * (size_t)(lv + 1) * n; z++) if (o[z] != o2[z]) return 3;
  }
  uint32_t gal[2] = {5, 2 * n - 1};
  uint32_t *evks = malloc(sizeof(uint32_t) * 2 * (size_t)dnum * 2 * el * n);
  uint32_t *outs = malloc(sizeof(uint32_t) * 2 * 2 * (size_t)nq * n);
  for (int r = 0; r < 2; r++) if (oracle_keygen_rotation(&p, m, 9 + r, gal[r], s, s2, evks + (size_t)r * dnum * 2 * el * n) < 0) return 4;
  if (oracle_rotate_hoisted(&p, m, nq - 1, d, d, 2, gal, evks, outs)) return 5;
  if (oracle_rotate_sum_hoisted(&p, m, nq - 1, d, d, 2, gal, evks, NULL, o)) return 6;
  if (oracle_mult_relin(&p, m, nq - 1, d, d, d, d, evk, o)) return 7;
  free(m); free(evk); free(d); free(o); free(o2); free(s); free(s2); free(evks); free(outs);
  return 0;
}
static int run64(uint32_t log_n, uint32_t nq, uint32_t dnum, uint32_t np) {
  oracle_params p = {log_n, nq, dnum, np};
  const uint32_t n = 1u << log_n, el = nq + np;
  uint64_t *m = malloc(sizeof(uint64_t) * el);
  uint64_t *evk = malloc(sizeof(uint64_t) * (size_t)dnum * 2 * el * n);
  uint64_t *d = malloc(sizeof(uint64_t) * (size_t)nq * n), *o = malloc(sizeof(uint64_t) * 2 * (size_t)nq * n);
  int8_t *s = malloc(n), *s2 = malloc(n);
  if (oracle64_moduli(&p, m) || oracle64_keygen(&p, m, 5, s, s2, evk) < 0) return 11;
  for (uint32_t i = 0; i < nq; i++) for (uint32_t z = 0; z < n; z++) d[(size_t)i * n + z] = ((uint64_t)z * 0x9e3779b97f4a7c15ull + i) % m[i];
  for (uint32_t lv = 0; lv < nq; lv++) if (oracle64_keyswitch(&p, m, lv, evk, d, o)) return 12;
  free(m); free(evk); free(d); free(o); free(s); free(s2);
  return 0;
}
int main(void) {
  int r;
  if ((r = run32(6, 4, 2, 2)) || (r = run32(7, 5, 2, 3)) || (r = run32(6, 7, 7, 1))) return r;
  if ((r = run64(6, 4, 2, 2)) || (r = run64(7, 5, 2, 3)) || (r = run64(6, 7, 7, 1))) return r;
  printf("oracle ok\n");
  return 0;
}
"""

NT_DRIVER = r"""
#include <cstdio>
#include "numtheory.h"
int main() {
  for (unsigned log_n = 12; log_n <= 17; log_n++) {
    unsigned p32[8];
    unsigned long long p64[8];
    if (ks::ntt_primes(log_n, 8, p32) || ks::ntt_primes64(log_n, 8, (uint64_t *)p64)) return 1;
    for (int i = 0; i < 8; i++)
      std::printf("%u %u %u %llu %llu\n", log_n, p32[i], ks::min_root_2n(p32[i], log_n), p64[i],
                  (unsigned long long)ks::min_root64(p64[i], log_n));
  }
  return 0;
}
"""


def _need(tool):
    if not shutil.which(tool):
        pytest.skip(f"no {tool}")


def test_oracle_under_asan_ubsan(tmp_path):
    _need("gcc")
    src = tmp_path / "drv.c"
    src.write_text(ORACLE_DRIVER)
    exe = tmp_path / "drv"
    od = os.path.join(ROOT, "oracle")
    subprocess.run(["gcc", "-std=c11", *SAN, "-I", od, str(src), os.path.join(od, "ks_oracle.c"),
                    os.path.join(od, "ks_oracle64.c"), "-o", str(exe), "-lm"], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600,
                       env={**os.environ, "ASAN_OPTIONS": "detect_leaks=1"})
    assert r.returncode == 0 and "oracle ok" in r.stdout, (r.returncode, r.stderr[-2000:])


def test_library_number_theory_under_asan_ubsan(tmp_path):
    _need("g++")
    src = tmp_path / "nt.cpp"
    src.write_text(NT_DRIVER)
    exe = tmp_path / "nt"
    cs = os.path.join(ROOT, "paper_2311_01598_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", *SAN, "-I", cs, str(src), os.path.join(cs, "numtheory.cpp"),
                    "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    rows = [list(map(int, line.split())) for line in r.stdout.splitlines()]
    assert len(rows) == 6 * 8
    for log_n in range(12, 18):
        got = [x for x in rows if x[0] == log_n]
        p32 = [int(v) for v in oracle.gen_primes(log_n, 8)]
        p64 = [int(v) for v in o64.gen_primes(log_n, 8)]
        assert [x[1] for x in got] == p32 and [x[3] for x in got] == p64
        for x in got[:2]:  # psi of both word sizes against the oracle
            assert x[2] == oracle.min_psi(x[1], log_n)
            assert x[4] == o64.min_psi(x[3], log_n)
