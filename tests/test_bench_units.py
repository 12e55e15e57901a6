"""The benchmark's per-product units (bench.py): RGSW bytes and modular
multiplications of one external product, for the default gadget (5 digits
of 6 bits per prime) against the MNIST-shaped figures the hot path's
definition fixes (N = 2048, two primes: 40 + 4 transforms, 659,456 modular
multiplications, 640 KiB of RGSW), and for 2 digits of 15 bits by counting
rows, transforms and multiply-accumulate terms one by one; and the kernel
code hash that guards the measured traffic ignores comments."""
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_default_gadget_mnist_figures(bench):
    assert bench.rgsw_bytes(2048, 2) == 640 * 1024
    assert bench.modmul_per_xp(2048, 2) == 659456


def count(N, nq, dig):
    """bytes and modular multiplications of one product, term by term"""
    rows = 2 * dig * nq                      # gadget rows of an RGSW (b side, then a side)
    nbytes = rows * 2 * nq * N * 4           # each row: an RLWE of 2 polynomials x nq residues
    fwd = 2 * nq * dig * nq                  # each digit polynomial of both input polynomials, at every prime
    inv = 2 * nq                             # the two output polynomials, at every prime
    butterflies = (N // 2) * (N.bit_length() - 1)
    mac = 0
    for _ in range(rows):                    # each digit polynomial times its row: 2 outputs x nq residues x N
        mac += 2 * nq * N
    return nbytes, (fwd + inv) * butterflies + mac


@pytest.mark.parametrize("N,nq", [(1024, 1), (2048, 2), (4096, 3), (2048, 3)])
@pytest.mark.parametrize("dig", [5, 2])
def test_units_by_counting(bench, N, nq, dig):
    nbytes, mm = count(N, nq, dig)
    assert bench.rgsw_bytes(N, nq, dig) == nbytes
    assert bench.modmul_per_xp(N, nq, dig) == mm


def test_two_digit_mnist_figures(bench):
    assert bench.rgsw_bytes(2048, 2, 2) == 262144
    assert bench.modmul_per_xp(2048, 2, 2) == 290816


def test_code_hash_ignores_comments(bench, tmp_path, monkeypatch):
    src = os.path.join(ROOT, "paper_2403_20190_amd", "csrc")
    base = tmp_path / "paper_2403_20190_amd" / "csrc"
    base.mkdir(parents=True)
    for f in bench.KERNEL_SOURCES:
        (base / f).write_text(open(os.path.join(src, f)).read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_code_sha256()
    f = base / bench.KERNEL_SOURCES[1]
    text = f.read_text()
    f.write_text("// a new comment line\n" + text.replace("\n", "  \n", 3) + "/* and a block\n comment */\n")
    assert bench.kernel_code_sha256() == h0
    f.write_text(text + "\nstatic const int added_code = 1;\n")
    assert bench.kernel_code_sha256() != h0
