"""lbm_device_copy, the bandwidth reference of the benchmark: both load kinds
copy every byte, at sizes that fill no whole workgroup, end mid-workgroup and
span many; misaligned or ragged arguments are refused on the host before any
launch."""
import pytest

from paper_1105_2904_amd import lbm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


@pytest.mark.parametrize("streaming", [True, False])
@pytest.mark.parametrize("nbytes", [16, 4096 + 16, (1 << 20) + 48, 3 << 24])
def test_copy_moves_every_byte(streaming, nbytes):
    import torch
    g = torch.Generator(device="cuda").manual_seed(nbytes)
    src = torch.randint(0, 256, (nbytes + 64,), dtype=torch.uint8, device="cuda", generator=g)
    dst = torch.zeros_like(src)
    stream = torch.cuda.current_stream()
    lbm.lbm_device_copy(dst.data_ptr(), src.data_ptr(), nbytes, stream.cuda_stream, streaming)
    torch.cuda.synchronize()
    assert torch.equal(dst[:nbytes], src[:nbytes])
    assert int(dst[nbytes:].count_nonzero()) == 0  # nothing past the end


def test_copy_refuses_bad_arguments():
    import torch
    src = torch.zeros(256, dtype=torch.uint8, device="cuda")
    dst = torch.zeros_like(src)
    s = torch.cuda.current_stream().cuda_stream
    for d, sp, n in ((dst.data_ptr() + 1, src.data_ptr(), 64), (dst.data_ptr(), src.data_ptr() + 8, 64),
                     (dst.data_ptr(), src.data_ptr(), 40)):
        with pytest.raises(lbm.LbmError):
            lbm.lbm_device_copy(d, sp, n, s)
    lbm.lbm_device_copy(dst.data_ptr(), src.data_ptr(), 0, s)  # nothing to do
