"""The level schedule (host code of the library) and the host builds under
AddressSanitizer / UndefinedBehaviorSanitizer, on the CPU.

* The library's schedule (irk_level_schedule, the one the factorization and
  the sweeps follow) against its definition, recomputed here by brute force
  from the pattern: forward level = 1 + the largest forward level of the
  lower neighbours (0 without), backward level the same over the upper
  neighbours (Sec. 4.2.1); every element listed once, ascending within a
  level.  Periodic 2D / 3D grids (permuted), a path in natural order (one
  element per level), isolated elements (one level), a complete bipartite
  mesh (rows longer than the sweep record).
* Patterns irk_setup must reject: malformed row pointers, columns out of
  range or out of order, a missing diagonal, an asymmetric pattern, a
  triangle.
* The same schedule code (csrc/schedule.h) compiled with g++
  -fsanitize=address,undefined into a small driver, run on the valid and
  the malformed patterns: no sanitizer report, and the same schedules.
* The oracle (oracle/oracle.c) compiled with the same sanitizers and
  loaded into a child Python process (libasan preloaded): a Radau IIA
  tableau, block ILU(0) factor and apply and a GMRES solve of each
  preconditioner on the small workload run without a report.
"""
import os
import shutil
import subprocess
import sys
import textwrap

import numpy as np
import pytest

import dgsynth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1701_07181_amd", "csrc")


def _irk():
    return pytest.importorskip("paper_1701_07181_amd")


def pattern(mesh, seed=None):
    """BSR pattern (row_ptr, col_idx) of a mesh, diagonal included, labels
    permuted by a seeded permutation when seed is given."""
    T = len(mesh)
    perm = np.random.default_rng(seed).permutation(T) if seed is not None else np.arange(T)
    rows = [None] * T
    for e in range(T):
        rows[int(perm[e])] = sorted({int(perm[e])} | {int(perm[f]) for f in mesh[e]})
    rp = np.zeros(T + 1, np.int32)
    for i in range(T):
        rp[i + 1] = rp[i] + len(rows[i])
    ci = np.array([j for r in rows for j in r], np.int32)
    return rp, ci


def bipartite(a, b):
    lo = b // 2
    hubs = list(range(lo, lo + a))
    leaves = [e for e in range(a + b) if e not in hubs]
    return [leaves if e in hubs else hubs for e in range(a + b)]


def reference_levels(rp, ci):
    """Levels by their definition (plain loops)."""
    T = len(rp) - 1
    lf = [0] * T
    for i in range(T):
        lower = [j for j in ci[rp[i]:rp[i + 1]] if j < i]
        lf[i] = 1 + max(lf[j] for j in lower) if lower else 0
    lb = [0] * T
    for i in range(T - 1, -1, -1):
        upper = [j for j in ci[rp[i]:rp[i + 1]] if j > i]
        lb[i] = 1 + max(lb[j] for j in upper) if upper else 0
    return lf, lb


def lists_from_levels(lev):
    L = max(lev) + 1
    lst = [i for l in range(L) for i in range(len(lev)) if lev[i] == l]
    off = [0]
    for l in range(L):
        off.append(off[-1] + sum(1 for x in lev if x == l))
    return np.array(lst, np.int32), np.array(off, np.int32)


VALID = {
    "grid2d_8": pattern(dgsynth.grid2d(8), seed=5),
    "grid2d_64": pattern(dgsynth.grid2d(64), seed=6),
    "grid3d_5": pattern(dgsynth.grid3d(5), seed=7),
    "path_30": pattern(dgsynth.path_mesh(30)),
    "isolated_9": pattern(dgsynth.isolated_mesh(9)),
    "bipartite_3_20": pattern(bipartite(3, 20)),
}


def _malformed():
    rp, ci = pattern(dgsynth.grid2d(4), seed=3)
    out = {}
    r = rp.copy(); r[0] = 1; out["rp0_nonzero"] = (r, ci)
    r = rp.copy(); r[5] = r[4] - 1; out["rp_decreasing"] = (r, ci)
    r = rp.copy(); r[-1] -= 1; out["rp_end_short"] = (r, ci)
    r = rp.copy(); r[3] = 1000; out["rp_past_end"] = (r, ci)
    c = ci.copy(); c[7] = 16; out["col_out_of_range"] = (rp, c)
    c = ci.copy(); c[rp[2]], c[rp[2] + 1] = c[rp[2] + 1], c[rp[2]]; out["cols_unsorted"] = (rp, c)
    # element 0 without its diagonal: drop the entry
    d = int(np.nonzero(ci[rp[0]:rp[1]] == 0)[0][0])
    c = np.delete(ci, d); r = rp.copy(); r[1:] -= 1; out["no_diagonal"] = (r, c)
    # asymmetric: 0 lists 2, 2 does not list 0 (a ring of 4 in natural order)
    ring = [[1, 3], [0, 2], [1, 3], [2, 0]]
    r4, c4 = pattern(ring)
    rows = [list(c4[r4[i]:r4[i + 1]]) for i in range(4)]
    rows[0] = sorted(set(rows[0]) | {2})
    rp2 = np.cumsum([0] + [len(x) for x in rows]).astype(np.int32)
    out["asymmetric"] = (rp2, np.array([j for x in rows for j in x], np.int32))
    # a triangle: 0-1, 1-2, 2-0
    out["triangle"] = pattern([[1, 2], [0, 2], [0, 1]])
    return out


MALFORMED = _malformed()


@pytest.mark.parametrize("name", list(VALID))
def test_level_schedule_matches_definition(name):
    irk = _irk()
    rp, ci = VALID[name]
    lf, of, lb, ob = irk.level_schedule(rp, ci)
    rf, rb = reference_levels(rp, ci)
    ef, eof = lists_from_levels(rf)
    eb, eob = lists_from_levels(rb)
    assert np.array_equal(lf, ef) and np.array_equal(of, eof)
    assert np.array_equal(lb, eb) and np.array_equal(ob, eob)
    T = len(rp) - 1
    if name == "path_30":
        assert len(of) - 1 == T and len(ob) - 1 == T     # one element per level
    if name == "isolated_9":
        assert len(of) - 1 == 1 and len(ob) - 1 == 1


@pytest.mark.parametrize("name", list(MALFORMED))
def test_level_schedule_rejects(name):
    irk = _irk()
    rp, ci = MALFORMED[name]
    with pytest.raises(irk.IrkError) as ei:
        irk.level_schedule(rp, ci)
    assert ei.value.status == irk.ERR_ARG


def _write_patterns(path, pats):
    with open(path, "w") as f:
        for rp, ci in pats:
            f.write(f"{len(rp) - 1} {len(ci)}\n")
            f.write(" ".join(str(int(x)) for x in rp) + "\n")
            f.write(" ".join(str(int(x)) for x in ci) + "\n")


def test_schedule_under_sanitizers(tmp_path):
    """schedule.h built with ASan + UBSan: valid and malformed patterns run
    without a report, with the library's statuses and schedules."""
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "sched_check")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-I", CSRC,
                    os.path.join(ROOT, "tests", "sched_check.cpp"), "-o", exe], check=True)
    names = list(VALID) + list(MALFORMED)
    pats = [VALID[n] for n in VALID] + [MALFORMED[n] for n in MALFORMED]
    inp = str(tmp_path / "patterns.txt")
    _write_patterns(inp, pats)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([exe, inp], capture_output=True, text=True, env=env, timeout=120)
    assert res.returncode == 0, res.stderr[-3000:]
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr
    lines = res.stdout.splitlines()
    k = 0
    for name in names:
        st = int(lines[k]); k += 1
        if name in MALFORMED:
            assert st == 1, name
            continue
        assert st == 0, name
        got = [np.array(lines[k + q].split(), np.int32) for q in range(4)]
        k += 4
        rp, ci = VALID[name]
        rf, rb = reference_levels(rp, ci)
        ef, eof = lists_from_levels(rf)
        eb, eob = lists_from_levels(rb)
        for g, e in zip(got, (ef, eof, eb, eob)):
            assert np.array_equal(g, e), name


def test_oracle_under_sanitizers(tmp_path):
    """oracle.c built with ASan + UBSan, driven from a child Python process."""
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    asan = subprocess.run([gcc, "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    if not asan or not os.path.exists(asan):
        pytest.skip("libasan not available")
    so = str(tmp_path / "liboracle_san.so")
    subprocess.run([gcc, "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-fPIC", "-shared",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-o", so, os.path.join(ROOT, "oracle", "oracle.c"), "-lm"], check=True)
    script = textwrap.dedent("""
        import os
        import numpy as np
        import dgsynth, oracle
        assert oracle.lib()._name == os.environ["IRK_ORACLE_LIB"]
        for s in range(1, 7):
            oracle.radau_iia(s)
        sy = dgsynth.config_system("cfg0")
        A, _, _ = oracle.radau_iia(sy.s)
        P = oracle.Problem(sy)
        v = np.random.default_rng(1).standard_normal(P.N)
        for pc in ("coupled", "uncoupled_shifted", "uncoupled"):
            oracle.pc_apply(P, A, pc, v)
            x, info = oracle.solve(P, A, sy.rhs, pc=pc, rtol=1e-10)
            assert info["converged"], (pc, info)
        oracle.matvec(P, oracle.inverse(A), v)
        print("ok")
    """)
    env = dict(os.environ, IRK_ORACLE_LIB=so, LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1",
               PYTHONPATH=ROOT + os.pathsep + os.environ.get("PYTHONPATH", ""))
    res = subprocess.run([sys.executable, "-c", script], capture_output=True, text=True, env=env,
                         cwd=ROOT, timeout=300)
    assert res.returncode == 0 and res.stdout.strip().endswith("ok"), res.stderr[-3000:]
    assert "runtime error" not in res.stderr
