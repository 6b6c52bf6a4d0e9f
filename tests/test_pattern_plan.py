"""Host checks of the general-pattern plan (no GPU): the C++ analysis in
csrc/pattern.hip is compiled with tests/pattern_plan_check.cpp and run on
structured-layout patterns (section 4's band, flow coupling and atom
columns) and random ones with dense rows and columns.  The checker verifies
table ranges, that the record layout and the transposed ELL hold every entry
once, and that LU without pivoting and the four triangular solves driven by
the plan's position tables reproduce dense elimination residuals."""
import os
import shutil
import subprocess

import pytest

from paper_2403_09198_amd import gen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not found")
    out = str(tmp_path_factory.mktemp("plan") / "check")
    cmd = [HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O1", "-std=c++17",
           f"-I{ROOT}/include", f"-I{ROOT}/paper_2403_09198_amd/csrc",
           f"{ROOT}/tests/pattern_plan_check.cpp", f"{ROOT}/paper_2403_09198_amd/csrc/pattern.hip",
           "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    return out


def _run(checker, patterns):
    lines = []
    for ip, ix in patterns:
        lines.append(f"{len(ip) - 1} {len(ix)} " + " ".join(map(str, ip)) + " " +
                     " ".join(map(str, ix)))
    r = subprocess.run([checker], input="\n".join(lines) + "\n0 0\n", capture_output=True,
                       text=True, timeout=120)
    return r.returncode, r.stdout.strip().split("\n")


def _fields(line):
    return dict(zip(("m", "nnz", "ne", "net", "ns", "nnzF"), map(int, line.split()[1:])))


@pytest.mark.parametrize("L", [2, 6, 61, 200])
def test_layout_patterns(checker, L):
    pats = [(b, a) for b in (1, 3, 8) for a in (0, 1, 2)]
    rc, out = _run(checker, [gen.layout_pattern(L, b, a) for b, a in pats])
    assert rc == 0, out
    assert all(o.startswith("ok") for o in out), out
    for (band, arrow), o in zip(pats, out):
        f = _fields(o)
        # a band needs no fill in the natural order and none after the ordering
        if arrow == 0:
            assert f["nnzF"] == f["nnz"], (band, o)
        # the flow unknowns (and the atom) become dense indices at any L
        # where their rows do not fit the ELL part
        if arrow and L > 16:
            assert f["ns"] >= 3, (band, arrow, o)
            assert f["ne"] <= 2 * band + 1, (band, arrow, o)


@pytest.mark.parametrize("m", [3, 11, 64, 65, 130, 256])
def test_random_patterns(checker, m):
    pats = [gen.random_pattern(m, per_row=3, dense_rows=(m // 2,), dense_cols=(1,), seed=s)
            for s in range(4)]
    pats.append(gen.random_pattern(m, per_row=min(m - 1, 6), seed=9))
    pats.append(gen.random_pattern(m, per_row=0, seed=1))  # diagonal only
    rc, out = _run(checker, pats)
    assert rc == 0, out
    assert all(o.startswith("ok") for o in out), out
    assert _fields(out[-1])["nnzF"] == m


def test_dense_and_malformed_patterns(checker):
    m = 12
    full = gen.random_pattern(m, per_row=m - 1, seed=0)   # every entry
    star = gen.random_pattern(m, per_row=0, dense_rows=(0,), dense_cols=(0,), seed=0)
    rc, out = _run(checker, [full, star])
    assert rc == 0 and out[0].startswith("ok") and out[1].startswith("ok"), out
    # a dense star in the natural order would fill everything; the ordering
    # puts its centre last and keeps the pattern
    assert _fields(out[1])["nnzF"] == _fields(out[1])["nnz"]
    ip, ix = gen.random_pattern(m, per_row=2, seed=1)
    no_diag = (ip, ix.copy())
    row0 = list(ix[ip[0]:ip[1]])
    no_diag[1][ip[0] + row0.index(0)] = [j for j in range(m) if j not in row0][0]
    dup = (ip, ix.copy())
    dup[1][ip[1] - 1] = dup[1][ip[0]]
    oob = (ip, ix.copy())
    oob[1][3] = m
    rc, out = _run(checker, [no_diag, dup, oob])
    assert [o.split()[0] for o in out] == ["ERR"] * 3, out
    assert "diagonal" in out[0] and "twice" in out[1] and "range" in out[2], out


def test_too_many_dense_indices_is_unsupported(checker):
    m = 40
    ip, ix = gen.random_pattern(m, per_row=2, dense_rows=tuple(range(0, 36, 2)), seed=3)
    rc, out = _run(checker, [(ip, ix)])
    assert out[0].startswith("ERR -7"), out
