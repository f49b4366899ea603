"""The measurement entry point: the plain streaming copy whose rate bench.py
reports as the HBM ceiling copies exactly, including a ragged tail past the
kernel's unrolled stride, and rejects what it cannot copy."""
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def yy():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1905_02300_amd import yy as mod
    mod.load()
    return mod


@pytest.mark.parametrize("n", [2, 1000, 2048 + 6, 3 * 256 * 16 * 256 + 6, (1 << 23) + (1 << 22) + 2])
def test_stream_copy_exact(yy, n):
    print(f"case: stream copy of {n} doubles", flush=True)
    g = torch.Generator(device="cuda").manual_seed(n)
    a = torch.rand(n, dtype=torch.float64, device="cuda", generator=g)
    b = torch.zeros_like(a)
    yy.stream_copy(b, a)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_stream_copy_rejects_bad_arguments(yy):
    print("case: stream copy argument checks", flush=True)
    a = torch.zeros(64, dtype=torch.float64, device="cuda")
    b = torch.zeros(64, dtype=torch.float64, device="cuda")
    with pytest.raises(yy.YYError) as e:
        yy.stream_copy(b[1:], a[1:])          # 8-byte aligned only
    assert e.value.status == yy.YY_ERR_ARG
    with pytest.raises(yy.YYError):
        yy.stream_copy(b[:3], a[:3])          # 24 bytes: not a multiple of 16
