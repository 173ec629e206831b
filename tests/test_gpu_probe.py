"""The HBM probe the benchmark reads its plain-streaming reference from:
rates within physical bounds on a buffer well beyond the caches, and its
argument checks."""
import pytest

from paper_2605_18052_amd import fastea

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_probe_rates_are_physical():
    read, copy = fastea.hbm_probe(0, 1 << 30, 3)
    print(f"HBM probe (1 GiB): read {read:.0f} GB/s, copy {copy:.0f} GB/s", flush=True)
    # below the 8 TB/s peak; above a quarter of it (a 1 GiB stream is 4x the
    # 256 MB Infinity Cache, so the rate is HBM's)
    assert 2000.0 < read < 8000.0
    assert 1000.0 < copy < 8000.0


def test_probe_rejects_bad_arguments():
    import ctypes as C
    r, c = C.c_double(0.0), C.c_double(0.0)
    L = fastea.lib()
    assert L.fea_hbm_probe(0, 1 << 10, 3, C.byref(r), C.byref(c)) == fastea.FEA_EINVAL  # under 1 MiB
    assert L.fea_hbm_probe(0, 1 << 24, 0, C.byref(r), C.byref(c)) == fastea.FEA_EINVAL  # no repetition
    assert L.fea_hbm_probe(0, 1 << 24, 1, None, C.byref(c)) == fastea.FEA_EINVAL
    assert L.fea_hbm_probe(-1, 1 << 24, 1, C.byref(r), C.byref(c)) == fastea.FEA_EINVAL
