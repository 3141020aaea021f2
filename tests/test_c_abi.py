"""The C interface used from a C program (tests/c/abi_example.c): both
headers compile as strict C99 and the program links against libflb.so; on
the CPU it checks that a rejected creation returns NULL with a message, on
the GPU that a whole run through the C calls gives the same results as the
same calls through the Python binding."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "c", "abi_example.c")
LIBDIR = os.path.join(ROOT, "paper_1010_1233_amd")


def _build(flb, tmp_path):
    exe = tmp_path / "abi_example"
    subprocess.run(["gcc", "-std=c99", "-pedantic", "-Wall", "-Wextra", "-Werror",
                    "-I", os.path.join(ROOT, "include"), "-o", str(exe), SRC,
                    "-L", LIBDIR, "-l:libflb.so", "-Wl,-rpath," + LIBDIR],
                   check=True, capture_output=True, text=True)
    return str(exe)


def test_c_program_compiles_links_and_sees_host_errors(flb, tmp_path):
    exe = _build(flb, tmp_path)
    r = subprocess.run([exe, "--invalid"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert "tau[3]" in r.stdout


@pytest.mark.gpu
def test_c_program_matches_the_binding(flb, tmp_path):
    exe = _build(flb, tmp_path)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    t, ns, checksum, mass, D, Q = r.stdout.split()
    g = flb.Lattice(48, 40, [1, 1, 1, 0.8, 0.8, 1.0, 1, 1, 1], 1e-4, u0=(0.05, 0.0), seed=7)
    g.thermalize()
    g.run(200, 10)
    acc, n = g.read_correlators()
    assert (int(t), int(ns)) == (g.t, n) == (200, 20)
    total = 0.0
    for v in acc.ravel().tolist():  # the C program's order
        total += v
    assert float(checksum) == total
    assert float(mass) == g.conservation()[0]
    assert (int(D), int(Q)) == (3, 15)
