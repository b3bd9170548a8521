"""A compression workspace carries the global range pass's slots from one
call to the next (left zero, and marked so). A workspace of arbitrary bytes,
one reused for fields of other sizes and element types, and one shared with
decompressions must all give the oracle's streams byte for byte: the first
call on unmarked bytes takes the path that does not trust the slots."""
import numpy as np
import pytest
import torch

from gpu_util import same_bits
from oracle import szref
from paper_2201_13020_amd import synth, szx


def _stream(out, size):
    n = int(size.cpu().view(torch.int64).item())
    assert n > 0
    return out[:n].cpu().numpy()


def _fields():
    rng = np.random.default_rng(13020 + 11)
    walk = np.cumsum(rng.standard_normal(300001)).astype(np.float64)
    return [
        ("sines 2^20 float32 REL 1e-3", synth.sines_1d(1 << 20), 1e-3, "rel"),
        ("turbulence 20x100x100 float32 REL 1e-4", synth.turbulence_3d((20, 100, 100)), 1e-4, "rel"),
        ("random walk 300001 float64 REL 1e-5", walk, 1e-5, "rel"),
        ("sines 2^16+37 float32 ABS 1e-3", synth.sines_1d((1 << 16) + 37), 1e-3, "abs"),
        ("sines 2^20 float32 REL 1e-2", synth.sines_1d(1 << 20, field=1), 1e-2, "rel"),
    ]


@pytest.mark.gpu
@pytest.mark.parametrize("fill", [0x00, 0xA5, 0xFF])
def test_reused_workspace_from_arbitrary_bytes(fill):
    fields = _fields()
    wsz = max(szx.workspace_size(torch.float32 if x.dtype == np.float32 else torch.float64, x.shape, eb, m, 128)
              for _, x, eb, m in fields)
    ws = torch.full((wsz,), fill, dtype=torch.uint8, device="cuda")
    refs = {name: szref.compress(x, eb, m, 128) for name, x, eb, m in fields}
    # twice over every field: the first call meets the fill bytes, the others
    # the slots the call before left (after fields of other sizes and types)
    for rnd in range(2):
        for name, x_np, eb, mode in fields:
            print(f"[workspace fill {fill:#x}] round {rnd}: {name}", flush=True)
            x = torch.from_numpy(x_np).cuda()
            out, size = szx.compress(x, eb, mode, 128, ws=ws)
            got = _stream(out, size)
            assert np.array_equal(got, refs[name]), name
            # a decompression through the same workspace in between
            y, st = szx.decompress(out, got.size, szx.inspect(got[:96].tobytes()), ws=ws)
            torch.cuda.synchronize()
            assert int(st.cpu().view(torch.int32).item()) == 0
            assert same_bits(y.cpu().numpy(), szref.decompress(refs[name]).ravel())


@pytest.mark.gpu
def test_workspace_unmarked_again_after_overwrite():
    """Overwriting the whole workspace (its first bytes included) between
    calls is allowed: the next call finds no mark and does not trust the
    slots."""
    x_np = synth.sines_1d(1 << 20)
    ref = szref.compress(x_np, 1e-3, "rel", 128)
    x = torch.from_numpy(x_np).cuda()
    ws = torch.empty(szx.workspace_size(torch.float32, x.shape, 1e-3, "rel", 128), dtype=torch.uint8,
                     device="cuda")
    for fill in (0x11, 0x00, 0xEE):
        out, size = szx.compress(x, 1e-3, "rel", 128, ws=ws)
        assert np.array_equal(_stream(out, size), ref)
        ws.fill_(fill)
        out, size = szx.compress(x, 1e-3, "rel", 128, ws=ws)
        assert np.array_equal(_stream(out, size), ref)


@pytest.mark.gpu
@pytest.mark.parametrize("fill", [0x00, 0xFF, 0x5A])
def test_decompression_clears_its_words_every_call(fill):
    """The index pass clears its look-back status words and the caller's
    status word itself, at every call (no launch of its own does): stale
    words between calls (all-ones words read as published prefixes), a
    stale error status, and a workspace of arbitrary bytes must not change a
    value or the status."""
    rng = np.random.default_rng(13020 + 12)
    walk = np.cumsum(rng.standard_normal((1 << 20) + 3)).astype(np.float64)
    fields = [("sines 2^22 float32 REL 1e-3", synth.sines_1d(1 << 22), 1e-3),
              ("random walk 2^20+3 float64 REL 1e-5", walk, 1e-5)]
    for name, x_np, eb in fields:
        ref = szref.compress(x_np, eb, "rel", 128)
        yref = szref.decompress(ref).ravel()
        exp = szx.inspect(ref[:96].tobytes())
        stream = torch.from_numpy(ref).cuda()
        tdt = torch.float32 if x_np.dtype == np.float32 else torch.float64
        ws = torch.full((szx.workspace_size(tdt, x_np.shape, eb, "rel", 128),), fill, dtype=torch.uint8,
                        device="cuda")
        st = torch.full((1,), 3, dtype=torch.uint32, device="cuda")
        for rnd in range(3):
            print(f"[decompression gate fill {fill:#x}] round {rnd}: {name}", flush=True)
            y, st = szx.decompress(stream, ref.size, exp, status=st, ws=ws)
            torch.cuda.synchronize()
            assert int(st.cpu().view(torch.int32).item()) == 0, (name, rnd)
            assert same_bits(y.cpu().numpy(), yref), (name, rnd)
            # everything past the gate's line dirtied again, and a stale status
            ws[256:].fill_(0xFF if rnd % 2 == 0 else fill)
            st.fill_(3)


@pytest.mark.gpu
def test_mixed_batch_decompression_clears_every_status():
    """A batch of both element types: the first index launch clears the
    statuses and status words of every field, the second finds its gate open;
    stale statuses between runs come back zero."""
    rng = np.random.default_rng(13020 + 13)
    xs = [synth.sines_1d(200_000 + 17 * i, field=i).astype(np.float64 if i % 3 == 0 else np.float32)
          for i in range(9)]
    refs = [szref.compress(x, 1e-3, "rel", 128) for x in xs]
    streams = [torch.from_numpy(r).cuda() for r in refs]
    exps = [szx.inspect(r[:96].tobytes()) for r in refs]
    d = szx.decompress_batch(streams, [r.size for r in refs], exps)
    for rnd in range(3):
        for s in d.statuses:
            s.fill_(int(rng.integers(1, 5)))
        d.run()
        torch.cuda.synchronize()
        for i, r in enumerate(refs):
            assert int(d.statuses[i].cpu().view(torch.int32).item()) == 0, (rnd, i)
            yref = szref.decompress(r).ravel()
            assert same_bits(d.outs[i][: yref.size].cpu().numpy(), yref), (rnd, i)
