"""Host-side checks of the C ABI library (no GPU needed).

The library loads, exports every entry point declared in include/ks.h, and
its own derivation of moduli and roots of unity agrees with the oracle's
independent one (trial division / brute-force root search).  Argument errors
that are decided before any device work return the documented status.
"""
import ctypes
import os
import re

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ks = pytest.importorskip("paper_2311_01598_amd")


def test_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "ks.h")).read()
    declared = set(re.findall(r"\b(ks(?:64)?_[a-z_]+)\s*\(", hdr))
    assert declared, "no declarations found"
    assert declared == set(ks.EXPORTS)
    for name in declared:
        assert hasattr(ks.lib(), name), name
    # the range-check build exports the same entry points
    check = ctypes.CDLL(os.path.join(os.path.dirname(ks.LIB_PATH), "libks_check.so"))
    for name in declared:
        assert hasattr(check, name), name


def test_range_checks_are_compiled_out_of_the_normal_build():
    if os.path.basename(ks.LIB_PATH) != "libks.so":
        pytest.skip("the range-check build is loaded")
    with pytest.raises(ks.KsError) as e:
        ks.ks_range_violations()
    assert e.value.status == ks.KS_ERR_UNSUPPORTED
    with pytest.raises(ks.KsError) as e:
        ks.ks_range_set_strict(True)
    assert e.value.status == ks.KS_ERR_UNSUPPORTED


@pytest.mark.parametrize("shape", [(12, 4, 2, 2), (16, 24, 3, 8), (14, 10, 3, 0), (17, 48, 3, 16), (15, 26, 3, 7)])
def test_moduli_match_oracle(shape):
    log_n, num_q, dnum, num_p = shape
    got = ks.ks_params_moduli(log_n, num_q, dnum, num_p)
    want = [int(x) for x in oracle.moduli(oracle.Params(log_n, num_q, dnum, num_p))]
    assert got == want


@pytest.mark.parametrize("log_n", [12, 14, 16, 17])
def test_roots_match_oracle(log_n):
    for q in oracle.gen_primes(log_n, 4):
        assert ks.ks_root_of_unity(int(q), log_n) == oracle.min_psi(int(q), log_n)


def test_root_rejects_bad_modulus():
    assert ks.ks_root_of_unity(1 << 30, 12) == 0            # not prime
    q = int(oracle.gen_primes(12, 1)[0])
    assert ks.ks_root_of_unity(q, 17) == 0 or (q - 1) % (2 << 17) == 0


def test_explicit_moduli_validation():
    good = ks.ks_params_moduli(12, 4, 2, 2)
    assert ks.ks_params_moduli(12, 4, 2, 2, moduli=good) == good
    bad_dup = list(good)
    bad_dup[1] = bad_dup[0]
    bad_comp = list(good)
    bad_comp[0] = good[0] + 2 * 4096   # same residue class, composite or not 2N-friendly prime
    for bad in (bad_dup, [m + 1 for m in good], [3] + good[1:]):
        with pytest.raises(ks.KsError) as e:
            ks.ks_params_moduli(12, 4, 2, 2, moduli=bad)
        assert e.value.status == ks.KS_ERR_INVALID_ARG


@pytest.mark.parametrize("shape,status", [((11, 4, 2, 2), "KS_ERR_UNSUPPORTED"), ((18, 4, 2, 2), "KS_ERR_UNSUPPORTED"),
                                          ((12, 0, 1, 1), "KS_ERR_INVALID_ARG"), ((12, 4, 5, 1), "KS_ERR_INVALID_ARG"),
                                          ((12, 4, 0, 1), "KS_ERR_INVALID_ARG"), ((16, 100, 1, 0), "KS_ERR_UNSUPPORTED")])
def test_plan_rejects_bad_params_before_device_work(shape, status):
    with pytest.raises(ks.KsError) as e:
        ks.ks_plan_create(*shape)
    assert e.value.status == getattr(ks, status)


def test_status_strings():
    for s in range(6):
        assert ks.ks_status_string(s)


def test_struct_layouts_match_the_header(tmp_path):
    """The Python binding's job and parameter structs have the header's
    sizes and field offsets (compiled here with the host C compiler)."""
    import ctypes
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if not cc:
        pytest.skip("no host C compiler")
    checks = {
        "ks_job_t": ["evk", "level", "in", "out"],
        "ks_seeded_job_t": ["evk_b", "a_seed", "level", "in", "out"],
        "ks_config_t": ["schedule", "tile_towers", "batch_mode", "spin_limit", "batch_order"],
        "ks_params_t": ["log_n", "num_q", "dnum", "num_p", "moduli"],
        "ks64_params_t": ["log_n", "num_q", "dnum", "num_p", "moduli"],
        "ks_rotation_t": ["evk", "galois", "out"],
        "ks_seeded_rotation_t": ["evk_b", "a_seed", "galois", "out"],
        "ks_rotation_term_t": ["evk", "galois", "diag"],
        "ks_rotate_job_t": ["evk", "galois", "level", "c0", "c1", "out"],
    }
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "ks.h"', "int main(void) {"]
    for t, fields in checks.items():
        lines.append(f'  printf("{t} %zu\\n", sizeof({t}));')
        for f in fields:
            lines.append(f'  printf("{t}.{f} %zu\\n", offsetof({t}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    r = subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src),
                        "-o", str(exe)], capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("header needs the HIP toolchain: " + r.stderr[-300:])
    got = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                        check=True).stdout.splitlines())
    pyname = {"in": "in_"}
    for t, fields in checks.items():
        cls = getattr(ks, t)
        assert int(got[t]) == ctypes.sizeof(cls), t
        for f in fields:
            assert int(got[f"{t}.{f}"]) == getattr(cls, pyname.get(f, f)).offset, (t, f)


def test_galois_rotation_matches_oracle():
    from oracle import core
    for log_n in (12, 16, 17):
        for r in (0, 1, 2, 5, -1, -7, (1 << log_n) // 2 - 1):
            assert ks.galois_rotation(log_n, r) == core.galois_rotation(log_n, r)
    assert ks.galois_rotation(12, 1) == 5


@pytest.mark.parametrize("shape", [(12, 4, 2, 2), (17, 45, 3, 15), (16, 24, 3, 8)])
def test_moduli64_and_roots_match_the_64bit_oracle(shape):
    """Host-only 64-bit-word calls: the library's moduli and psi equal the
    64-bit oracle's (derived independently: generator method in the
    library, quadratic non-residue in the oracle)."""
    from oracle import core64 as o64
    log_n, num_q, dnum, num_p = shape
    mods = ks.ks64_params_moduli(log_n, num_q, dnum, num_p)
    assert mods == [int(v) for v in o64.moduli(oracle.Params(log_n, num_q, dnum, num_p))]
    for q in (mods[0], mods[-1]):
        assert ks.ks64_root_of_unity(q, log_n) == o64.min_psi(q, log_n)
    assert ks.ks64_root_of_unity(mods[0] + 2, log_n) == 0
    with pytest.raises(ks.KsError):
        ks.ks64_params_moduli(log_n, num_q, dnum, num_p, moduli=[(1 << 30) + 1] * (num_q + (num_p or num_q)))
