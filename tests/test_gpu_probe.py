"""The roofline probes run, report their work, and are deterministic."""
import pytest

from paper_1902_05234_amd import aes
from tests.gpu_util import cuda

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("which", [aes.AES_PROBE_LDS, aes.AES_PROBE_VALU])
def test_probe_runs_and_is_deterministic(which):
    torch = cuda()
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    out = torch.zeros(cus * 2048, dtype=torch.int32, device="cuda")
    work = aes.aes_roof_probe(which, 50, out)
    assert work == cus * 2048 * 16 * 50
    first = out.clone()
    aes.aes_roof_probe(which, 50, out)
    torch.cuda.synchronize()
    assert torch.equal(first, out)
    with pytest.raises(aes.AesError):
        aes.aes_roof_probe(which, 50, out[:100])      # too small for one word per probe thread
