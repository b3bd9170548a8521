"""Stream files through device memory: a compressed stream written to a file
and loaded back is byte-identical and decompresses to the oracle's values;
sizes around the staging chunk (16 MiB) and host/device mixes round-trip."""
import numpy as np
import pytest

from oracle import szref
from gpu_util import same_bits

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


CHUNK = 16 << 20


def test_dump_and_load_a_compressed_stream(tmp_path):
    from paper_2201_13020_amd import szx, synth
    x = synth.batch_field(dict(dims=(300, 1000), dtype="float32", eb=1e-3, zero_regions=True, seed=31), "cuda")
    out, size = szx.compress(x, 1e-3, "rel", 128, dims=(300, 1000))
    n = int(size.cpu().view(torch.int64).item())
    p = str(tmp_path / "field.szx")
    szx.file_write(p, out, nbytes=n, durable=True)  # ordered after the compression, no sync needed
    assert szx.file_size(p) == n
    back, got = szx.file_read(p)
    assert got == n and torch.equal(back[:n], out[:n])
    ref = szref.compress(x.cpu().numpy(), 1e-3, "rel", 128)
    assert np.array_equal(back[:n].cpu().numpy(), ref)
    y, st = szx.decompress(back, n, dict(dtype=torch.float32, dims=(300, 1000), block=128))
    torch.cuda.synchronize()
    assert int(st.cpu().view(torch.int32).item()) == 0
    assert same_bits(y.cpu().numpy(), szref.decompress(ref))


@pytest.mark.parametrize("nbytes", [1, 4097, CHUNK - 1, CHUNK, CHUNK + 1, 2 * CHUNK + 12345])
def test_sizes_around_the_staging_chunk(tmp_path, nbytes):
    from paper_2201_13020_amd import szx
    print(f"[io] {nbytes} bytes", flush=True)
    g = torch.Generator(device="cuda").manual_seed(nbytes)
    d = torch.randint(0, 256, (nbytes + 7,), dtype=torch.uint8, device="cuda", generator=g)
    p = str(tmp_path / f"b{nbytes}")
    szx.file_write(p, d, nbytes=nbytes)
    assert szx.file_size(p) == nbytes
    with open(p, "rb") as f:
        assert f.read() == d[:nbytes].cpu().numpy().tobytes()
    dst = torch.full((nbytes + 64,), 0xAB, dtype=torch.uint8, device="cuda")
    _, got = szx.file_read(p, out=dst)
    assert got == nbytes and torch.equal(dst[:nbytes], d[:nbytes])
    assert bool((dst[nbytes:] == 0xAB).all()), "bytes past the file were written"


def test_host_and_device_mixes(tmp_path):
    from paper_2201_13020_amd import szx
    h = torch.arange(3 * CHUNK // 8 + 5, dtype=torch.int64)  # pageable host memory
    p = str(tmp_path / "host")
    szx.file_write(p, h)
    dev, got = szx.file_read(p)
    assert got == h.numel() * 8 and torch.equal(dev[:got].view(torch.int64).cpu(), h)
    p2 = str(tmp_path / "dev")
    szx.file_write(p2, dev, nbytes=got)
    back = torch.empty_like(h)
    _, got2 = szx.file_read(p2, out=back)
    assert got2 == got and torch.equal(back, h)
