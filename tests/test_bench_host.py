"""Host-side checks of bench.py's bookkeeping (no GPU needed).

The algorithmic byte and multiply counts of the Output-Centric stages are
checked against hand counts of the bench workload (N = 2^16, l+1 = 24,
dnum 3, K = 8), and the traffic-counter digest ignores comments but not code.
"""
import os
import shutil

import bench


def test_stage_bytes_hand_count():
    limb = 4 << 16
    b = bench.stage_bytes(16, 24, 8, 8)
    # xt in, ycol out: 24 + 3 digits x (8 special + 16 foreign) targets
    assert b["oc.bconv_col.up"] == limb * (24 + 3 * 24)
    # ycol of 2 foreign digits, 2 ModDown terms, d, key 3 x 2, out 2 (per Q tower)
    assert b["oc.row.q"] == limb * 24 * (2 + 2 + 1 + 6 + 2)
    # ycol of 3 digits, key 3 x 2, 2 outputs (per special tower)
    assert b["oc.row.p"] == limb * 8 * (3 + 6 + 2)
    assert b["oc.row.q.seeded"] == b["oc.row.q"] - limb * 24 * 3  # the a halves are regenerated
    assert sum(v for k, v in b.items() if "seeded" not in k) == 180355072


def test_stage_muls_hand_count():
    n = 1 << 16
    m = bench.stage_muls(16, 24, 8, 8)
    row_pass = 3 * 8 * n // 2          # 8 stages of N/2 Shoup butterflies, 3 multiplies each
    assert m["oc.intt_row"] == 24 * row_pass
    col_pass = 3 * 8 * n // 2
    # every (digit, target) pair: 8 multiply-accumulates + REDC (4) per word, then a column pass
    assert m["oc.bconv_col.up"] == 3 * 24 * (n * (8 + 4) + col_pass)


def test_alg_bytes_is_input_key_output():
    n = 1 << 16
    assert bench.alg_bytes(n, 24, 8, 3) == 4 * n * (24 + 2 * 3 * 32 + 2 * 24)


def test_source_digest_ignores_comments_not_code(tmp_path):
    src = os.path.join(bench.ROOT, "paper_2311_01598_amd", "csrc")
    a = tmp_path / "a"
    shutil.copytree(src, a)
    base = bench.kernel_source_digest(str(a))
    assert base == bench.kernel_source_digest()
    f = a / "oc_kernels.h"
    text = f.read_text()
    f.write_text(text.replace("namespace ks {", "// a new remark\nnamespace ks {  /* and another */", 1))
    assert bench.kernel_source_digest(str(a)) == base
    f.write_text(text.replace("constexpr int kPad = 272;", "constexpr int kPad = 276;", 1))
    assert bench.kernel_source_digest(str(a)) != base
    f.write_text(text)
    # a code edit in a compile unit outside the 32-bit key switch leaves it
    g = a / "ks64.hip"
    g.write_text(g.read_text().replace("constexpr uint32_t kList = 96;", "constexpr uint32_t kList = 64;", 1))
    assert bench.kernel_source_digest(str(a)) == base


def test_batch_bytes_count_the_shared_key_once():
    n = 1 << 16
    # 16 key switches sharing one key: 16 x (6 MiB in + 12 MiB out) + one 48 MiB key
    assert bench.batch_alg_bytes(n, 24, 8, 3, 16) == 16 * (18 << 20) + (48 << 20)
    assert bench.batch_alg_bytes(n, 24, 8, 3, 1) == bench.alg_bytes(n, 24, 8, 3)
