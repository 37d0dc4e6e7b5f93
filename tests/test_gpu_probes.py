"""The measurement probes through the C-ABI (include/mlmc_probe.h): every gather mode
(device memory or LDS-staged table, independent streams or one serial stream per lane) and
the integer VALU probe launch, report the work they did, and take a positive time. Their
rates calibrate the rooflines and are not asserted here."""
import sys

import pytest
import torch

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_1904_12754_amd import api as _api
    return _api


@pytest.mark.parametrize("lds", [False, True])
@pytest.mark.parametrize("dependent", [False, True])
def test_gather_probe_modes(api, lds, dependent):
    log2, waves, iters = 11, 8, 16
    table = torch.zeros((16 << log2) // 4, dtype=torch.int32, device="cuda")
    g, s = api.probe_gather(table, log2, waves, iters, lds=lds, dependent=dependent)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    lanes = cus * waves * 64
    _say(f"lds={lds} dependent={dependent}: {g} gathers in {s * 1e6:.1f} us ({g / s:.3e}/s)")
    assert g == lanes * iters * (1 if dependent else 8)
    assert s > 0.0


def test_gather_probe_refuses_an_lds_table_past_64kb(api):
    table = torch.zeros((16 << 13) // 4, dtype=torch.int32, device="cuda")
    with pytest.raises(Exception):
        api.probe_gather(table, 13, 8, 4, lds=True)


def test_valu_probe(api):
    n, s = api.probe_valu(8, 64)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    assert n == cus * 8 * 64 * 64 * 8 and s > 0.0
