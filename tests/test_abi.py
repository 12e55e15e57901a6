"""CPU checks of the C ABI: the library loads and exports every function the
header declares (no device work is issued)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hwisard.h")
LIB = os.path.join(ROOT, "paper_2403_20190_amd", "libhwisard.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hw_[a-z0-9_]+)\s*\(", src)))


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhwisard.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    names = declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhwisard.so not built")
def test_binding_covers_header():
    from paper_2403_20190_amd import hwisard as HW
    assert set(declared()) <= set(HW.exported_symbols())


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhwisard.so not built")
def test_host_only_calls():
    """Calls that never touch the device: permutation parity with the oracle
    and argument checks that fail before anything is enqueued."""
    import numpy as np

    import oracle as O
    from paper_2403_20190_amd import hwisard as HW
    for s, seed in [(1, 3), (2, 5), (128, 9), (2352, 11), (4704, 12)]:
        assert np.array_equal(HW.permutation(HW.shape(s, 2, 8, seed)), O.permutation(seed, s))
    with pytest.raises(HW.HwError):
        HW.permutation(HW.shape(0, 2, 8, 1))


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhwisard.so not built")
def test_tune_variant_names():
    """The tuned kernels and their variant tables (host only)."""
    from paper_2403_20190_amd import hwisard as HW
    counts = {"train": 8, "infer": 4, "train_batch": 2, "infer_batch": 2, "ntt": 4, "ntt_inverse": 4,
              "encrypt_rgsw": 3}
    assert set(counts) == set(HW.TUNED_KERNELS)
    for k, n in counts.items():
        names = [HW.tune_variant_name(k, v) for v in range(n)]
        assert all(names) and len(set(names)) == n
        assert HW.tune_variant_name(k, n) is None and HW.tune_variant_name(k, -1) is None
    assert HW.tune_variant_name("xp", 0) is None


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhwisard.so not built")
def test_request_seeds_match_oracle():
    """The serving engine's per-request seeds (host only): the library and the
    oracle derive them with their own generators; the input and label seeds
    of one request differ, and neighbouring enc_seed values share no seed."""
    import oracle as O
    from paper_2403_20190_amd import hwisard as HW
    seen = set()
    for e in [0, 1, 2, 500, 501, 8000, 8001, 2**63 + 5, 2**64 - 1]:
        sx, sy = HW.request_seeds(e)
        assert (sx, sy) == O.request_seeds(e)
        assert sx != sy and sx not in seen and sy not in seen
        seen.update((sx, sy))
