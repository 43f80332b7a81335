"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and its host-only calls (defaults, Algorithm 1 schedule, CSR
validation, transpose check, row binning statistics) behave.  No GPU needed."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2510_24429_amd import _lib as L
from paper_2510_24429_amd import lpgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pdhg.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pdhg_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    lib = L.lib()
    names = header_functions()
    assert len(names) >= 30
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(L.SIGNATURES), set(names) ^ set(L.SIGNATURES)


def test_noalloc_scratch_size_matches_header():
    text = open(HEADER).read()
    m = re.search(r"#define PDHG_SPMV_NOALLOC_MAX_BYTES \(\(size_t\)(\d+) << (\d+)\)", text)
    assert m, "PDHG_SPMV_NOALLOC_MAX_BYTES not found"
    assert int(m.group(1)) << int(m.group(2)) == L.SPMV_NOALLOC_MAX_BYTES


def test_struct_layouts_match_header(tmp_path):
    # compile a probe against the header and compare every field offset with
    # the ctypes mirror
    structs = {"pdhg_params": L.Params, "pdhg_kkt": L.KKT, "pdhg_info": L.Info,
               "pdhg_snapshot_info": L.SnapInfo,
               "pdhg_refine_params": L.RefineParams,
               "pdhg_refine_info": L.RefineInfo,
               "pdhg_kernel_time": L.KernelTime}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pdhg.h"',
             'int main(void) {']
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    import subprocess
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src),
                           "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    for line in out:
        if not line:
            continue
        cname, field, val = line.split()
        py = structs[cname]
        if field == "size":
            assert C.sizeof(py) == int(val), cname
        else:
            assert getattr(py, field).offset == int(val), (cname, field)


def test_param_defaults():
    p, _ = L.default_params()
    assert (p.ruiz_passes, p.power_iters, p.eval_every) == (10, 100, 64)
    assert p.eps_rel == 1e-6 and p.eta_factor == 0.9
    assert (p.beta_suff, p.beta_nec, p.beta_art, p.omega_theta) == (0.2, 0.8, 0.36, 0.5)


def _golden():
    out = []
    with open(os.path.join(ROOT, "tests", "golden", "alg1_schedule.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                lhs, rhs = line.split(":")
                out.append((*map(float, lhs.split()), [float(t) for t in rhs.split()]))
    return out


@pytest.mark.parametrize("ec,er,expect", _golden())
def test_alg1_levels_match_paper(ec, er, expect):
    got = L.alg1_levels(ec, er)
    assert len(got) == len(expect)
    assert np.allclose(got, expect, rtol=1e-15, atol=0)


def _validate(rows, cols, rp, ci):
    rp = np.asarray(rp, dtype=np.int64)
    ci = np.asarray(ci, dtype=np.int32)
    msg = C.create_string_buffer(256)
    rc = L.lib().pdhg_validate_csr(rows, cols, int(rp[-1]),
                                   rp.ctypes.data_as(C.c_void_p),
                                   ci.ctypes.data_as(C.c_void_p), msg, 256)
    return rc, msg.value.decode()


def test_validate_csr():
    assert _validate(2, 3, [0, 2, 3], [0, 2, 1])[0] == 0
    rc, msg = _validate(2, 3, [0, 2, 1, 3][:3], [0, 2, 1])
    assert rc == -2
    rc, msg = _validate(2, 3, [0, 2, 3], [0, 3, 1])
    assert rc == -2 and "out of range" in msg
    rc, msg = _validate(2, 3, [0, 2, 3], [2, 0, 1])
    assert rc == -2 and "increasing" in msg
    rc, msg = _validate(2, 3, [0, 2, 3], [1, 1, 1])
    assert rc == -2
    rc, msg = _validate(2, 3, [1, 2, 3], [0, 1, 2])
    assert rc == -2


def _check_t(lp, at_v=None, at_ci=None):
    perm = np.zeros(lp.nnz, dtype=np.int64)
    msg = C.create_string_buffer(256)
    arrs = [lp.a_rp, lp.a_ci, lp.a_v, lp.at_rp,
            lp.at_ci if at_ci is None else at_ci,
            lp.at_v if at_v is None else at_v]
    rc = L.lib().pdhg_check_transpose(lp.m, lp.n, lp.nnz,
                                      *[a.ctypes.data_as(C.c_void_p) for a in arrs],
                                      perm.ctypes.data_as(C.c_void_p), msg, 256)
    return rc, perm, msg.value.decode()


def test_transpose_check_and_permutation():
    lp = lpgen.planted_powerlaw(m=300, n=2000, kmax=200, seed=3)
    rc, perm, _ = _check_t(lp)
    assert rc == 0
    assert np.array_equal(perm, lp.a_perm_to_at())
    bad = lp.at_v.copy()
    bad[17] = np.nextafter(bad[17], np.inf)          # one ulp: bitwise check
    rc, _, msg = _check_t(lp, at_v=bad)
    assert rc == -3 and "transpose" in msg
    badc = lp.at_ci.copy()
    j = int(np.argmax(np.diff(lp.at_rp) >= 2))
    p = lp.at_rp[j]
    badc[p], badc[p + 1] = badc[p + 1], badc[p]     # unsorted row
    rc, _, _ = _check_t(lp, at_ci=badc)
    assert rc == -2


def test_loading_without_gpu_reports_device_error():
    # creating a context needs a GPU; on a CPU-only machine the call must fail
    # cleanly with an error code rather than crash
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    ctx = C.c_void_p()
    rc = L.lib().pdhg_create(0, None, C.byref(ctx))
    assert rc < 0 and not ctx.value


def _plan(rp, tile, thr, chunk):
    rp = np.ascontiguousarray(rp, dtype=np.int64)
    cap = 4 * len(rp) + 1000
    out = np.zeros(4 * cap, dtype=np.int32)
    k = L.lib().pdhg_plan_bins(len(rp) - 1, rp.ctypes.data_as(C.c_void_p), tile,
                               thr, chunk, out.ctypes.data_as(C.c_void_p), cap)
    assert k > 0
    return out[:4 * k].reshape(k, 4)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_row_bins_cover_every_row_once(seed):
    rng = np.random.default_rng(seed)
    lens = np.concatenate([np.zeros(30, dtype=np.int64), rng.integers(1, 20, 3000),
                           rng.integers(20, 1100, 300), rng.integers(1100, 9000, 30),
                           np.array([50_000, 123_457])])
    rng.shuffle(lens)
    rp = np.concatenate([[0], np.cumsum(lens)])
    tile, thr, chunk = 1021, 40_000, 10_000
    blk = _plan(rp, tile, thr, chunk)
    covered = np.zeros(len(lens), dtype=np.int64)
    seen_long = True
    for r0, r1, part, nparts in blk:
        assert 0 <= r0 < r1 <= len(lens)
        if r1 - r0 > 1 or nparts == 1:
            if part == 0:
                covered[r0:r1] += 1
        nz = rp[r1] - rp[r0]
        if r1 - r0 > 1:
            seen_long = False
            assert nz <= tile and r1 - r0 <= tile      # fits the LDS tile
        else:
            assert seen_long or lens[r0] <= tile     # long rows come first
            if nparts > 1:
                assert lens[r0] > thr and nparts == -(-lens[r0] // chunk)
                if part == 0:
                    covered[r0] += 1
    assert np.all(covered == 1)
    # split parts of one row are all present, in order
    for row in np.nonzero(lens > thr)[0]:
        parts = blk[(blk[:, 0] == row) & (blk[:, 3] > 1)][:, 2]
        assert list(parts) == list(range(len(parts)))


# ---------------------------------------------------------------- panels

def _plan_panels(rp, ci, cols, P, cut, tile=1021):
    rp = np.ascontiguousarray(rp, dtype=np.int64)
    ci = np.ascontiguousarray(ci, dtype=np.int32)
    cut = np.ascontiguousarray(cut, dtype=np.int64)
    rows = len(rp) - 1
    srp = np.zeros(P * rows + 1, dtype=np.int64)
    src = np.zeros(max(len(ci), 1), dtype=np.int32)
    cap = 8 * (P * rows + 8) + 1000
    out = np.zeros(4 * cap, dtype=np.int32)
    vp = lambda a: a.ctypes.data_as(C.c_void_p)
    k = L.lib().pdhg_plan_panels(rows, cols, vp(rp), vp(ci), P, vp(cut), tile,
                                 vp(srp), vp(src), vp(out), cap)
    assert k > 0, k
    return srp, src[:len(ci)], out[:4 * k].reshape(k, 4)


@pytest.mark.parametrize("P", [1, 2, 4, 8])
def test_column_panels_partition_every_row(P):
    rng = np.random.default_rng(P)
    lp = lpgen.planted_powerlaw(m=3000, n=9000, kmax=700, seed=P)
    rows, cols = lp.m, lp.n
    cut = np.array([cols * p // P for p in range(P + 1)], dtype=np.int64)
    if P > 2:                       # uneven cuts too
        cut[1] = cut[1] // 3
    srp, src, blk = _plan_panels(lp.a_rp, lp.a_ci, cols, P, cut)
    # stacked row p*rows+i = row i's entries with column in panel p, in order
    assert srp[0] == 0 and srp[-1] == lp.nnz and np.all(np.diff(srp) >= 0)
    assert np.array_equal(np.sort(src), np.arange(lp.nnz))
    for i in rng.integers(0, rows, 200):
        cols_i = lp.a_ci[lp.a_rp[i]:lp.a_rp[i + 1]]
        for p in range(P):
            s0, s1 = srp[p * rows + i], srp[p * rows + i + 1]
            want = cols_i[(cols_i >= cut[p]) & (cols_i < cut[p + 1])]
            assert np.array_equal(lp.a_ci[src[s0:s1]], want)
    # blocks: every non-empty stacked row exactly once (empty ones at most
    # once: no block starts at one), a block never leaves its panel, and the
    # block at launch index w serves panel (w % 8) % P
    covered = np.zeros(P * rows, dtype=np.int64)
    for w, (r0, r1, part, nparts) in enumerate(blk):
        if r0 == r1:
            continue
        p = r0 // rows
        assert (r1 - 1) // rows == p and (w % 8) % P == p
        assert nparts == 1
        covered[r0:r1] += 1
        assert srp[r0 + 1] > srp[r0]
        if r1 - r0 > 1:
            assert srp[r1] - srp[r0] <= 1021
    nonempty = np.diff(srp) > 0
    assert np.all(covered[nonempty] == 1) and np.all(covered[~nonempty] <= 1)
    # XCD queues hold whole rows of the 8-wide launch grid
    assert len(blk) % 8 == 0


def test_column_panels_reject_int32_overflow():
    # P * rows stacked rows must stay below 2^31; only sizes are read before
    # the check, so tiny arrays stand in for a matrix of 2^29 rows
    rp = np.zeros(2, dtype=np.int64)
    ci = np.zeros(1, dtype=np.int32)
    cut = np.array([0, 1, 2, 3, 4, 5, 6, 7, 8], dtype=np.int64)
    srp = np.zeros(2, dtype=np.int64)
    src = np.zeros(1, dtype=np.int32)
    vp = lambda a: a.ctypes.data_as(C.c_void_p)
    rc = L.lib().pdhg_plan_panels(1 << 28, 8, vp(rp), vp(ci), 8, vp(cut), 1021,
                                  vp(srp), vp(src), None, 0)
    assert rc == -1


def test_column_panels_skip_empty_runs():
    # block-diagonal rows: each row's entries lie in one panel, so 3 of its 4
    # stacked rows are empty; blocks must cover the non-empty ones once and
    # leave the long empty runs alone
    rng = np.random.default_rng(7)
    rows, cols, P = 4000, 4000, 4
    rp = np.arange(rows + 1, dtype=np.int64) * 5
    ci = np.concatenate([np.sort(rng.choice(1000, 5, replace=False)) + 1000 * (i // 1000)
                         for i in range(rows)]).astype(np.int32)
    cut = np.array([0, 1000, 2000, 3000, 4000], dtype=np.int64)
    srp, src, blk = _plan_panels(rp, ci, cols, P, cut)
    nonempty = np.diff(srp) > 0
    assert nonempty.sum() == rows
    covered = np.zeros(P * rows, dtype=np.int64)
    for r0, r1, part, nparts in blk:
        covered[r0:r1] += 1
    assert np.all(covered[nonempty] == 1)
    # each panel's run of non-empty rows ends in at most one block that
    # reaches into the following empty run
    assert covered.sum() <= rows + P * 1021


def test_panel_choice_follows_table_size():
    # gather tables that fit one XCD's L2 stay whole; an 8 MB table over
    # long rows is split; short rows over a huge table pay too much in
    # partial sums for a small table split
    assert L.lib().pdhg_choose_panels(200_000, 200_000, 9_400_000) == 1
    assert L.lib().pdhg_choose_panels(200_000, 1_000_000, 9_400_000) > 1
    assert L.lib().pdhg_choose_panels(1_350_000, 4_950_000, 14_550_000) == 8
    assert L.lib().pdhg_choose_panels(5_000_000, 20_000_000, 110_000_000) == 8
    assert L.lib().pdhg_choose_panels(20_000_000, 5_000_000, 110_000_000) == 4
    # ~3 entries per row: splitting the 10.8 MB table costs more than it saves
    assert L.lib().pdhg_choose_panels(4_950_000, 1_350_000, 14_550_000) == 1
    assert L.lib().pdhg_choose_panels(100, 100, 0) == 1
    assert L.lib().pdhg_choose_panels(0, 10, 10) < 0
