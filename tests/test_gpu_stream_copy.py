"""The library's streaming copy kernel (the HBM reference the pixel-wise
roofline is read against): the destination equals the source, for both access
widths, on sizes that leave a ragged tail of the grid-stride loop."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("width", [16, 8])
@pytest.mark.parametrize("nbytes", [16, 4096 + 48, (1 << 24) + 16 * 37])
def test_stream_copy_copies(width, nbytes):
    import torch
    import paper_2010_07284_amd as vlg
    ctx = vlg.create(0)
    g = torch.Generator(device="cpu").manual_seed(nbytes + width)
    src = torch.randint(0, 256, (nbytes,), generator=g, dtype=torch.uint8).to("cuda:0")
    dst = torch.zeros_like(src)
    ms = vlg.stream_copy(ctx, dst, src, width=width, reps=2)
    assert ms > 0
    assert torch.equal(dst, src)


def test_stream_copy_rejects_width_that_does_not_divide():
    import torch
    import paper_2010_07284_amd as vlg
    ctx = vlg.create(0)
    a = torch.zeros(24, dtype=torch.uint8, device="cuda:0")
    b = torch.zeros_like(a)
    with pytest.raises(vlg.VlgError):
        vlg.stream_copy(ctx, b, a, width=16)
    with pytest.raises(vlg.VlgError):
        vlg.stream_copy(ctx, b, a, width=4)
