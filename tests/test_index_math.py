"""CPU check of the kernels' index arithmetic (periodic and walled).

The neighbour offsets of every stage and solver kernel come from
paper_2205_05835_amd/csrc/tpf_index.hpp.  The kernels do not clamp them (a
debug build with TPF_BOUNDS_CLAMP does), so their correctness rests on this
test: tests/index_check.cpp includes that same header, compiled for the host
with g++, and checks every cell of odd, ragged, 2-cell and workload-sized
grids against the wrapped coordinates (and, with free-slip walls on any set
of axes, against the mirrored ones), plus the XCD block -> tile map.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2205_05835_amd", "csrc")

GRIDS = [
    (2, 2, 1), (2, 2, 2), (3, 2, 1), (33, 21, 1), (15, 12, 10), (70, 24, 16), (24, 16, 10),
    (7, 6, 5), (128, 4, 1), (1, 1, 1), (5, 1, 3), (64, 64, 64), (96, 48, 32), (192, 192, 1),
    (129, 65, 9), (256, 256, 16),
]


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("idx") / "index_check")
    src = os.path.join(ROOT, "tests", "index_check.cpp")
    subprocess.run(["g++", "-O2", "-std=c++17", "-Wall", "-I", CSRC, "-o", exe, src], check=True)
    return exe


def test_offsets_and_tiles_match_wrapped_coordinates(checker):
    args = [str(v) for g in GRIDS for v in g]
    r = subprocess.run([checker, *args], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok")


def test_checker_catches_a_wrong_offset(checker, tmp_path):
    """The check itself must fail on a planted mistake: a copy of the header
    with the lower x offset of the first column made non-periodic."""
    src = open(os.path.join(CSRC, "tpf_index.hpp")).read()
    bad = src.replace("C.o[0][0] = i == 0 ? nx - 1 : -1;", "C.o[0][0] = -1;")
    assert bad != src
    d = tmp_path / "bad"
    d.mkdir()
    (d / "tpf_index.hpp").write_text(bad)
    exe = str(tmp_path / "index_check_bad")
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", str(d), "-o", exe,
                    os.path.join(ROOT, "tests", "index_check.cpp")], check=True)
    r = subprocess.run([exe, "33", "21", "1"], capture_output=True, text=True)
    assert r.returncode == 1 and "MISMATCH off" in r.stdout


def test_checker_catches_a_wrong_wall_offset(checker, tmp_path):
    """A planted mistake in the wall rule (the upper wall read periodically)
    must fail the wall check."""
    src = open(os.path.join(CSRC, "tpf_index.hpp")).read()
    bad = src.replace("if (v[a] == n[a] - 1) C.wl |= 2u << (4 * a);", "")
    assert bad != src
    d = tmp_path / "badw"
    d.mkdir()
    (d / "tpf_index.hpp").write_text(bad)
    exe = str(tmp_path / "index_check_badw")
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", str(d), "-o", exe,
                    os.path.join(ROOT, "tests", "index_check.cpp")], check=True)
    r = subprocess.run([exe, "6", "5", "1"], capture_output=True, text=True)
    assert r.returncode == 1 and "MISMATCH wall" in r.stdout
