"""Batched path: many fields of mixed element types, sizes and bounds in one
launch per pass. Every field's stream must equal the single-call stream and
the oracle's, byte for byte; decoded values bit for bit; graph replays and
other launch geometries must not change a byte."""
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


def make_fields(seed, count):
    from paper_2201_13020_amd import synth
    r = np.random.default_rng(seed)
    fields = []
    for i in range(count):
        kind = i % 5
        n = int(r.integers(1, 300_000)) if kind else int(r.integers(0, 3))
        dt = np.float64 if r.random() < 0.3 else np.float32
        if kind == 4 and n >= 64:
            x = synth.turbulence_3d((4, 4, n // 16), field=i).astype(dt)
        else:
            x = synth.sines_1d(max(n, 1), field=i)[:n].astype(dt)
        if kind == 3 and n > 10:
            x[n // 2] = np.nan
        eb = [1e-2, 1e-3, 1e-4, 0.0][int(r.integers(0, 4))]
        mode = "rel" if r.random() < 0.8 else "abs"
        fields.append((x, eb, mode))
    return fields


def test_batch_matches_single_and_oracle():
    from paper_2201_13020_amd import szx
    fields = make_fields(1, 40)
    xs = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x, _, _ in fields]
    b = szx.compress_batch(xs, [f[1] for f in fields], [f[2] for f in fields], 128,
                           dims=[x.shape if x.ndim else (1,) for x, _, _ in fields])
    for geom in [None, (8, None), (77, "f32"), (3, "f64"), (1, None), (4096, None)]:
        if geom:
            b.set_geometry(*geom)
        for o in b.outs:
            o.fill_(0xAB)
        b.run()
        torch.cuda.synchronize()
        for i, (x, eb, mode) in enumerate(fields):
            n = int(b.sizes[i].cpu().view(torch.int64).item())
            got = b.outs[i][:n].cpu().numpy()
            ref = szref.compress(x, eb, mode, 128)
            assert n == ref.size and np.array_equal(got, ref), f"field {i} geometry {geom}"
    # decompress the batch's own streams as a batch
    exps = [szx.inspect(b.outs[i][:96].cpu().numpy().tobytes()) for i in range(len(fields))]
    nb = [int(s.cpu().view(torch.int64).item()) for s in b.sizes]
    d = szx.decompress_batch(b.outs, nb, exps)
    d.run()
    torch.cuda.synchronize()
    for i, (x, eb, mode) in enumerate(fields):
        assert int(d.statuses[i].cpu().view(torch.int32).item()) == 0, i
        yref = szref.decompress(szref.compress(x, eb, mode, 128)).ravel()
        assert same_bits(d.outs[i][: yref.size].cpu().numpy(), yref), f"field {i}"


def test_batch_graph_replays():
    from paper_2201_13020_amd import szx
    fields = make_fields(2, 24)
    xs = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x, _, _ in fields]
    b = szx.compress_batch(xs, [f[1] for f in fields], [f[2] for f in fields], 128)
    b.run()
    torch.cuda.synchronize()
    ref = [b.outs[i][: int(b.sizes[i].cpu().view(torch.int64).item())].cpu().numpy().copy() for i in range(len(xs))]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.run()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.run()
    for rep in range(3):
        for o in b.outs:
            o.zero_()
        g.replay()
        torch.cuda.synchronize()
        for i in range(len(xs)):
            n = ref[i].size
            assert int(b.sizes[i].cpu().view(torch.int64).item()) == n
            assert np.array_equal(b.outs[i][:n].cpu().numpy(), ref[i]), f"replay {rep} field {i}"
        other = torch.from_numpy(make_fields(3, 1)[0][0].astype(np.float32)).cuda()
        szx.compress(other, 1e-3, "rel", 128)
        torch.cuda.synchronize()


def test_batch_rejects_mixed_block_sizes():
    from paper_2201_13020_amd import szx
    xs = [torch.zeros(100, device="cuda"), torch.zeros(100, device="cuda")]
    p0 = szx.make_params(torch.float32, (100,), 1e-3, "rel", 128)
    p1 = szx.make_params(torch.float32, (100,), 1e-3, "rel", 64)
    arr = (szx.SzCField * 2)()
    arr[0].params, arr[1].params = p0, p1
    assert szx.lib().sz_batch_workspace_size(arr, None, 2) == 0


def _batch_vs_oracle(specs, device_gen, sample=None, progress=lambda m: None):
    """Batch-compress the spec fields, check every stream against the oracle
    (or a sample of them), then batch-decompress and check values and the
    bound on every field."""
    from paper_2201_13020_amd import synth, szx
    xs = [synth.batch_field(sp, "cuda" if device_gen else "cpu").cuda() for sp in specs]
    progress(f"generated {len(xs)} fields")
    ebs = [sp["eb"] for sp in specs]
    b = szx.compress_batch(xs, ebs, "rel", 128, dims=[sp["dims"] for sp in specs])
    b.run()
    torch.cuda.synchronize()
    lens = torch.stack(b.sizes).cpu().view(torch.int64).reshape(-1).tolist()
    heads = torch.stack([o[:96] for o in b.outs]).cpu().numpy()
    exps = [szx.inspect(h.tobytes()) for h in heads]
    d = szx.decompress_batch(b.outs, lens, exps)
    d.run()
    torch.cuda.synchronize()
    st = torch.stack(d.statuses).cpu().view(torch.int32).reshape(-1)
    assert int(st.abs().sum()) == 0
    progress("batch compress and decompress done")
    check = range(len(xs)) if sample is None else sample
    for i in check:
        xh = xs[i].cpu().numpy()
        ref = szref.compress(xh, ebs[i], "rel", 128)
        got = b.outs[i][:lens[i]].cpu().numpy()
        assert lens[i] == ref.size and np.array_equal(got, ref), f"field {i} {specs[i]}"
        yref = szref.decompress(ref).ravel()
        assert same_bits(d.outs[i][: yref.size].cpu().numpy(), yref), f"field {i} values"
    progress(f"{len(check)} fields equal the oracle")
    # the bound on every field (a property that holds at any size): with e the
    # header's bound, fl(|x - x'|) <= e follows from the exact |x - x'| <= e
    for i, x in enumerate(xs):
        e_bits = int(np.frombuffer(heads[i][64:72].tobytes(), dtype=np.uint64)[0])
        e = float(np.array([e_bits], dtype=np.uint64).view(np.float64)[0]) if x.dtype == torch.float64 else \
            float(np.array([e_bits & 0xFFFFFFFF], dtype=np.uint32).view(np.float32)[0])
        y = d.outs[i][: x.numel()]
        err = (x.reshape(-1).double() - y.double()).abs().max().item() if x.numel() else 0.0
        assert err <= e, f"field {i}: error {err} above bound {e}"
    return b, d, xs, lens


def test_batch_of_many_uneven_fields_small():
    """The many-field workload at reduced sizes (96 fields, median 64 KiB):
    every stream and value equal to the oracle's."""
    from paper_2201_13020_amd import synth
    specs = synth.batch_specs(96, median=64 << 10, hi=2 << 20)
    _batch_vs_oracle(specs, device_gen=False)


@pytest.mark.slow
def test_batch_of_4096_fields_full(capsys):
    """The full many-field workload (4096 fields, about 8.8 GiB): every batch
    stream equal to the single-call stream, a random sample of fields equal
    to the oracle, every field within its bound."""
    from paper_2201_13020_amd import synth, szx

    def progress(msg):
        with capsys.disabled():
            print(f"[batch] {msg}", flush=True)

    specs = synth.batch_specs(4096)
    r = np.random.default_rng(11)
    sample = sorted(r.choice(4096, size=24, replace=False).tolist())
    b, d, xs, lens = _batch_vs_oracle(specs, device_gen=True, sample=sample, progress=progress)
    progress(f"{len(xs)} fields, {sum(x.numel() * x.element_size() for x in xs) / 2**30:.2f} GiB: batch matches")
    for i, x in enumerate(xs):
        o, s = szx.compress(x, specs[i]["eb"], "rel", 128, dims=specs[i]["dims"])
        torch.cuda.synchronize()
        assert int(s.cpu().view(torch.int64).item()) == lens[i]
        assert torch.equal(o[:lens[i]], b.outs[i][:lens[i]]), f"field {i}"
        del o, s
        if i % 1024 == 1023:
            progress(f"single calls equal the batch for fields 0..{i}")
