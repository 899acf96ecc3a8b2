"""The library's streaming copy, the bandwidth reference of the measurements:
it moves exactly the bytes asked for (several workgroups and a partial last
one, a single word), leaves the bytes after them untouched, and rejects a
size that is not whole 16-byte words."""
import pytest

from gpu_common import banner
from paper_2511_01629_amd import lbm

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("words", [1, 255, 256 * 3 + 5])
def test_copy_exact(words):
    banner(f"copy {words} words")
    import torch

    nbytes = 16 * words
    g = torch.Generator().manual_seed(words)
    src = torch.randint(0, 256, (nbytes + 64,), dtype=torch.uint8, generator=g).cuda()
    dst = torch.zeros(nbytes + 64, dtype=torch.uint8, device="cuda")
    st = torch.cuda.current_stream()
    lbm.copy(dst.data_ptr(), src.data_ptr(), nbytes, st.cuda_stream)
    torch.cuda.synchronize()
    assert torch.equal(dst[:nbytes], src[:nbytes])
    assert not dst[nbytes:].any()


def test_copy_rejects_partial_words():
    banner("copy partial word")
    import torch

    a = torch.zeros(64, dtype=torch.uint8, device="cuda")
    b = torch.zeros(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(lbm.LbmError) as e:
        lbm.copy(b.data_ptr(), a.data_ptr(), 40, torch.cuda.current_stream().cuda_stream)
    assert e.value.code == lbm.LBM_EINVAL


@pytest.mark.parametrize("narrays,words", [(9, 256 * 3 + 5), (19, 300), (3, 257), (1, 1)])
def test_copy_arrays_exact(narrays, words):
    """The multi-array copy (the Q-stream bandwidth reference) moves every
    array exactly and nothing beyond the last one."""
    banner(f"copy_arrays {narrays} x {words} words")
    import torch

    per = 16 * words
    nbytes = narrays * per
    g = torch.Generator().manual_seed(narrays * 1000 + words)
    src = torch.randint(0, 256, (nbytes + 64,), dtype=torch.uint8, generator=g).cuda()
    dst = torch.zeros(nbytes + 64, dtype=torch.uint8, device="cuda")
    st = torch.cuda.current_stream()
    lbm.copy_arrays(dst.data_ptr(), src.data_ptr(), narrays, per, st.cuda_stream)
    torch.cuda.synchronize()
    assert torch.equal(dst[:nbytes], src[:nbytes])
    assert not dst[nbytes:].any()
