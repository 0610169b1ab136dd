"""AddressSanitizer + UndefinedBehaviorSanitizer builds of the CPU oracle and
of the library's host code (no GPU needed).

- The oracle (plain C) is compiled with gcc and both sanitizers and run over
  ordinary and malformed inputs; every result must equal the ordinary
  build's (oracle.rcm) and the run must report nothing.
- Every library source is compiled by hipcc with the sanitizers on its host
  code only (each -fsanitize= behind -Xarch_host) and linked with
  tests/native/host_checks.cpp, whose checks exercise the host paths that
  run without a GPU: argument and option validation, the tuning-table parser
  on good and malformed tables, workspace sizes, the abort-flag registry,
  the server's configuration checks and the shuffle bijection.

Builds are cached under _build/sanitize/<hash of the sources>."""

import hashlib
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from paper_1610_08128_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1610_08128_amd", "csrc")
NATIVE = os.path.join(ROOT, "tests", "native")
INCLUDE = os.path.join(ROOT, "include")
HIPCC = "/opt/rocm/bin/hipcc"
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:halt_on_error=1",
           "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}


def _digest(paths):
    h = hashlib.sha256()
    for p in sorted(paths):
        h.update(p.encode())
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _build_dir(tag, sources):
    d = os.path.join(ROOT, "_build", "sanitize", f"{tag}-{_digest(sources)}")
    os.makedirs(d, exist_ok=True)
    return d


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    if r.returncode != 0:
        raise AssertionError(f"{' '.join(cmd)}\nexit {r.returncode}\n{r.stdout[-3000:]}\n"
                             f"{r.stderr[-6000:]}")
    return r


# ---------------------------------------------------------------------------
# The oracle
# ---------------------------------------------------------------------------

def _oracle_binary():
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    srcs = [os.path.join(ROOT, "oracle", "rcm_oracle.c"), os.path.join(NATIVE, "oracle_checks.c")]
    d = _build_dir("oracle", srcs)
    exe = os.path.join(d, "oracle_checks")
    if not os.path.exists(exe):
        _run(["gcc", "-O1", "-g", "-std=c99", "-Wall", "-Wextra",
              "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
              "-fno-omit-frame-pointer", "-o", exe + ".tmp"] + srcs)
        os.replace(exe + ".tmp", exe)
    return exe


def _cases():
    """(graph arrays, pp_variant, reverse_mode, full_check, cm_mode)."""
    out = []
    graphs = [I.grid2d(9, 13, seed=1), I.grid3d(4, 5, 3, seed=2), I.rgg_patches(400, 3),
              I.path(17, seed=4), I.star(12), I.cycle(9), I.complete(6),
              I.disjoint_union([I.grid2d(5, 6), I.path(4), I.star(5), I.path(1)], seed=5),
              I.shuffle_rows(I.drop_diagonal(I.grid2d(7, 8, seed=6)), 7),
              I.random_tree(60, 8), I.erdos_renyi(50, 0.08, 9)]
    for i, g in enumerate(graphs):
        for pp in (0, 1):
            for cm in (0, 1, 2, 3):
                out.append((g.n, g.rowptr, g.colidx, pp, (i + cm) % 2, 1, cm))
    # empty, single vertex, isolated vertices only
    out.append((0, np.zeros(1, np.int32), np.zeros(0, np.int32), 0, 0, 0, 0))
    out.append((1, np.array([0, 0], np.int32), np.zeros(0, np.int32), 0, 0, 1, 0))
    out.append((5, np.zeros(6, np.int32), np.zeros(0, np.int32), 1, 1, 1, 1))
    # malformed patterns (rowptr[n] is always the entry count given)
    g = I.grid2d(4, 5)
    rp, ci = g.rowptr.copy(), g.colidx.copy()
    bad = []
    x = rp.copy(); x[0] = 1; bad.append((x, ci))                       # rowptr[0] != 0
    x = rp.copy(); x[5], x[6] = x[6], x[5]; bad.append((x, ci))        # decreasing rowptr
    y = ci.copy(); y[7] = g.n; bad.append((rp, y))                     # column out of range
    y = ci.copy(); y[3] = -1; bad.append((rp, y))                      # negative column
    y = ci.copy(); y[rp[2] + 1] = y[rp[2]]; bad.append((rp, y))        # duplicate in a row
    for r_, c_ in bad:
        out.append((g.n, r_, c_, 0, 0, 0, 0))
    # asymmetric: one entry of a symmetric pair moved
    a = I.path(6, diag=False)
    ca = a.colidx.copy()
    ca[0] = 3  # (0,1) becomes (0,3), (1,0) stays
    out.append((a.n, a.rowptr, ca, 0, 0, 1, 0))
    out.append((a.n, a.rowptr, ca, 0, 0, 0, 0))
    return out


def _write_cases(path, cases):
    with open(path, "wb") as f:
        for n, rp, ci, pp, rev, full, cm in cases:
            rp = np.ascontiguousarray(rp, np.int32)
            ci = np.ascontiguousarray(ci, np.int32)
            assert rp.size == n + 1 and int(rp[-1]) == ci.size
            np.array([n, ci.size, pp, rev, full, cm], np.int32).tofile(f)
            rp.tofile(f)
            ci.tofile(f)


def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    exe = _oracle_binary()
    cases = _cases()
    path = str(tmp_path / "cases.bin")
    _write_cases(path, cases)
    r = _run([exe, path], env={**os.environ, **SAN_ENV,
                               "ASAN_OPTIONS": "detect_leaks=1:halt_on_error=1"}, timeout=300)
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-3000:]
    lines = r.stdout.splitlines()
    assert len(lines) == len(cases)
    statuses = []
    for line, (n, rp, ci, pp, rev, full, cm) in zip(lines, cases):
        want = oracle.rcm(n, rp, ci, pp_variant=pp, reverse_mode=rev, full_check=bool(full),
                          cm_mode=cm)
        head, _, tail = line.partition(" ")
        status = int(head)
        statuses.append(status)
        assert status == want.status, (n, pp, rev, full, cm)
        if status != oracle.OK:
            continue
        left, _, right = tail.partition("|")
        vals = [int(v) for v in left.split()]
        st = dict(zip(oracle.STAT_FIELDS, vals[:9]))
        assert st == want.stats
        assert np.array_equal(np.array(vals[9:], np.int64), want.perm)
        assert np.array_equal(np.array([int(v) for v in right.split()], np.int64), want.iperm)
    # the malformed and asymmetric inputs really took the error paths
    assert statuses.count(oracle.ERR_BAD_CSR) == 5
    assert statuses.count(oracle.ERR_NOT_SYMMETRIC) == 1


# ---------------------------------------------------------------------------
# The library's host code
# ---------------------------------------------------------------------------

SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def _host_binary():
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not found")
    lib_srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))
    headers = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp"))
    headers += sorted(os.path.join(INCLUDE, f) for f in os.listdir(INCLUDE) if f.endswith(".h"))
    driver = os.path.join(NATIVE, "host_checks.cpp")
    d = _build_dir("host", lib_srcs + headers + [driver])
    exe = os.path.join(d, "host_checks")
    if os.path.exists(exe):
        return exe
    common = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-I" + INCLUDE, "-I" + CSRC] + SAN_FLAGS

    def compile_one(src):
        obj = os.path.join(d, os.path.basename(src) + ".o")
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        _run(common + lang + ["-c", src, "-o", obj])
        return obj

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, lib_srcs + [driver]))
    _run([HIPCC, "--offload-arch=gfx950"] + SAN_FLAGS + ["-o", exe + ".tmp"] + objs +
         ["-pthread"])
    os.replace(exe + ".tmp", exe)
    return exe


def test_library_host_code_under_address_and_undefined_sanitizers(tmp_path):
    exe = _host_binary()
    # the HIP runtime keeps allocations until exit, so leak checking is off;
    # heap overflows, use after free and undefined behaviour still abort
    r = _run([exe, str(tmp_path)], env={**os.environ, **SAN_ENV}, timeout=300)
    assert "runtime error" not in r.stderr, r.stderr[-3000:]
    assert r.stdout.strip().endswith(", 0 failed"), r.stdout + r.stderr[-3000:]
    checks = int(r.stdout.split()[0])
    assert checks > 150
