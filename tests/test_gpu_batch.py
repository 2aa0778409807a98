"""GPU tests of the batched search and the device generator (needs an MI355X).

* the persistent, graph-captured batch gives results bitwise equal to one plain
  launch per cube, on every graph replay (with eager work in between);
* on small host-generated cubes the batch matches the FP64 oracle;
* at the benchmarked size (64 uneven cubes, ~108 GB) graph replay equals plain
  launches bit for bit, and the smallest cube matches the oracle in full;
* every row copy of the batch kernel (16- and 4-byte global-to-LDS loads,
  ordinary loads for odd 16-bit rows and misaligned cubes) equals plain launches;
* the device Philox4x32-10 words equal the host implementation bit for bit,
  and its Box-Muller normals agree with an FP64 evaluation.
"""
import numpy as np
import pytest

from oracle.delays import delay_table
from paper_2510_18136_amd import nsfrb, synth
from tests._lib import ensure_built
from tests.test_gpu_search import compare, oracle_run, to_device

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

C1_DMS = np.linspace(0, 1000, 8)
C1_W = [1, 2, 4, 8, 16]


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_built()
    assert torch.cuda.is_available()


def test_philox_words_match_host():
    n = 50_000
    out = torch.zeros(4 * n, dtype=torch.int32, device="cuda")
    print("[gpu] philox fill", flush=True)
    nsfrb.philox_fill(out.data_ptr(), n, 0x123456789ABCDEF, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    dev = out.cpu().numpy().view(np.uint32)
    assert np.array_equal(dev, synth.philox_blocks(n, 0x123456789ABCDEF))


@pytest.mark.parametrize("dtype", ["f32", "f16"])
def test_device_noise_matches_fp64_box_muller(dtype):
    n = 1 << 20
    tdt = torch.float32 if dtype == "f32" else torch.float16
    out = torch.empty(n, dtype=tdt, device="cuda")
    nsfrb.generate_noise(out.data_ptr(), dtype, "pst", n, 1, 1, seed=77, sigma=1.5,
                         stream=torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    got = out.float().cpu().numpy().astype(np.float64)
    ref = synth.philox_normals(n, 77, sigma=1.5)
    tol = 5e-5 * np.maximum(1, np.abs(ref)) if dtype == "f32" else 2e-3 * np.maximum(1, np.abs(ref))
    assert (np.abs(got - ref) <= tol).all()
    assert abs(got.mean()) < 0.01 and abs(got.std() - 1.5) < 0.01


def uneven_cfgs(rng, n, layout, store):
    cfgs = []
    for i in range(n):
        side = int(rng.choice([8, 16, 24, 40]))
        ns = int(rng.choice([8, 16]))
        nt = int(rng.choice([64, 100, 256, 300, 600]))
        cfgs.append(nsfrb.SearchConfig(side, side, nt, np.linspace(1.311, 1.499, ns), C1_DMS, C1_W,
                                       in_dtype=store, store_dtype=store,
                                       norm="none" if layout == "pst" else "pixel_subband",
                                       layout=layout, snr_threshold=5.0, max_candidates=16))
    return cfgs


def results(b, n):
    out = []
    for i in range(n):
        snr, toa = b.maps(i)
        cands, ntot = b.candidates(i)
        out.append((snr, toa, cands, ntot))
    return out


def same(a, b):
    for (s1, t1, c1, n1), (s2, t2, c2, n2) in zip(a, b):
        assert np.array_equal(s1, s2, equal_nan=True) and np.array_equal(t1, t2)
        assert c1 == c2 and n1 == n2


def test_batch_graph_replays_equal_separate_launches():
    rng = np.random.default_rng(4)
    cfgs = uneven_cfgs(rng, 9, "pst", "f16")
    stream = torch.cuda.current_stream()
    cubes = []
    for i, c in enumerate(cfgs):
        x = torch.empty(c.n_pix * c.n_sub * c.n_time, dtype=torch.float16, device="cuda")
        nsfrb.generate_noise(x.data_ptr(), "f16", "pst", c.n_pix, c.n_sub, c.n_time, seed=1000 + i,
                             stream=stream.cuda_stream)
        off = delay_table(c.freqs, c.freqs.max(), 134.2, [500.0])[0]
        nsfrb.inject_boxcar(x.data_ptr(), "f16", "pst", c.n_pix, c.n_sub, c.n_time, pixel=c.n_pix // 2, t0=20,
                            width=4, amp=3.0, offsets=off, stream=stream.cuda_stream)
        cubes.append(x)
    ptrs = [x.data_ptr() for x in cubes]
    print(f"[gpu] batch of {len(cfgs)} cubes", flush=True)
    with nsfrb.Batch(cfgs) as b:
        b.run_separate(ptrs, stream.cuda_stream)
        ref = results(b, len(cfgs))
        for rep in range(3):
            junk = torch.randn(1 << 20, device="cuda").sum().item()          # eager work between replays
            b.run(ptrs, stream.cuda_stream)
            got = results(b, len(cfgs))
            assert b.info()["graph"]
            same(got, ref)
        b.use_graph(False)
        b.run(ptrs, stream.cuda_stream)
        same(results(b, len(cfgs)), ref)
        info = b.info()
        assert info["work_items"] > 0 and info["classes"] >= 1
    # every cube's pulse is found at its pixel
    for i, (snr, toa, cands, ntot) in enumerate(ref):
        assert ntot >= 1 and cands[0]["x"] + cfgs[i].nx * cands[0]["y"] == cfgs[i].n_pix // 2


def test_batch_matches_oracle_on_small_cubes():
    rng = np.random.default_rng(8)
    cfgs = uneven_cfgs(rng, 5, "tsp", "f32")
    stream = torch.cuda.current_stream()
    host, dev = [], []
    for i, c in enumerate(cfgs):
        cube = synth.noise_cube(c.n_time, c.n_sub, c.n_pix, seed=50 + i)
        off = delay_table(c.freqs, c.freqs.max(), 134.2, [428.0])[0]
        synth.inject_boxcar(cube, 3, 30, off, 8, 2.5)
        host.append(cube)
        dev.append(to_device(cube, "f32"))
    with nsfrb.Batch(cfgs) as b:
        print("[gpu] batch vs oracle", flush=True)
        b.run([x.data_ptr() for x in dev], stream.cuda_stream)
        for i, c in enumerate(cfgs):
            snr, toa = b.maps(i)
            cands, ntot = b.candidates(i)
            o = oracle_run(host[i], c)
            fin = np.isfinite(o["snr_max"])
            assert np.array_equal(np.isfinite(snr), fin)
            assert np.abs(snr[fin] - o["snr_max"][fin]).max() <= 1e-4
            clear = fin & (o["margin"] > 2e-4)
            assert np.array_equal(toa[clear], o["toa"][clear])
            assert ntot == o["n_total"]


def test_batch_row_copies_of_every_alignment():
    """The persistent batch copies a cube's rows into LDS with 16-byte or 4-byte
    global-to-LDS loads, or with ordinary loads (16-bit rows of odd length, or a
    cube that starts off a 4-byte boundary): every path gives maps and
    candidates bitwise equal to one plain launch per cube, and the odd cube
    matches the oracle."""
    widths = [1, 2, 4, 8, 16]
    cases = [(16, 8, 256, 0), (16, 8, 100, 0), (8, 16, 101, 0), (8, 8, 64, 1), (24, 16, 333, 0)]
    stream = torch.cuda.current_stream().cuda_stream
    cfgs, cubes, views = [], [], []
    for k, (side, ns, nt, shift) in enumerate(cases):
        c = nsfrb.SearchConfig(side, side, nt, np.linspace(1.311, 1.499, ns), C1_DMS, widths, in_dtype="f16",
                               store_dtype="f16", norm="none", layout="pst", snr_threshold=5.0, max_candidates=16)
        n = side * side * ns * nt
        x = torch.empty(n + 8, dtype=torch.float16, device="cuda")
        v = x[shift:shift + n]                       # shift 1: a cube 2 bytes past an aligned address
        nsfrb.generate_noise(v.data_ptr(), "f16", "pst", side * side, ns, nt, 700 + k, stream=stream)
        off = delay_table(c.freqs, c.freqs.max(), 134.2, [500.0])[0]
        nsfrb.inject_boxcar(v.data_ptr(), "f16", "pst", side * side, ns, nt, pixel=side * side // 2, t0=20,
                            width=4, amp=2.0, offsets=off, stream=stream)
        cfgs.append(c)
        cubes.append(x)
        views.append(v)
    ptrs = [v.data_ptr() for v in views]
    assert ptrs[3] % 4 == 2
    print(f"[gpu] batch row copies: {len(cfgs)} cubes", flush=True)
    with nsfrb.Batch(cfgs) as b:
        b.run_separate(ptrs, stream)
        ref = results(b, len(cfgs))
        b.use_graph(False)
        b.run(ptrs, stream)
        same(results(b, len(cfgs)), ref)
        b.use_graph(True)
        b.run(ptrs, stream)
        same(results(b, len(cfgs)), ref)
    k = 2
    c = cfgs[k]
    z = views[k].cpu().numpy().astype(np.float32).reshape(c.n_pix, c.n_sub, c.n_time)
    o = oracle_run(np.transpose(z, (2, 1, 0)).copy(), c)
    snr, toa, cands, ntot = ref[k]
    fin = np.isfinite(o["snr_max"])
    assert np.array_equal(np.isfinite(snr), fin)
    assert np.abs(snr[fin] - o["snr_max"][fin]).max() <= 2e-4
    clear = fin & (o["margin"] > 2e-4)
    np.testing.assert_array_equal(toa[clear], o["toa"][clear])
    assert ntot == o["n_total"]


@pytest.mark.parametrize("pix", [1, 2, 4])
def test_batch_pixels_per_item(monkeypatch, pix):
    """Work items of 1, 2 or 4 pixels (NSFRB_BATCH_PIX), on cubes whose pixel
    counts are odd (the last item of a cube runs past it): maps, per-pixel best
    and candidates bitwise equal to one plain launch per cube."""
    monkeypatch.setenv("NSFRB_BATCH_PIX", str(pix))
    widths = [1, 2, 4, 8, 16]
    cases = [(7, 5, 8, 256), (9, 9, 16, 100), (13, 3, 8, 333), (4, 4, 16, 64)]
    stream = torch.cuda.current_stream().cuda_stream
    cfgs, cubes = [], []
    for k, (nx, ny, ns, nt) in enumerate(cases):
        c = nsfrb.SearchConfig(nx, ny, nt, np.linspace(1.311, 1.499, ns), C1_DMS, widths, in_dtype="f16",
                               store_dtype="f16", norm="none", layout="pst", snr_threshold=5.0, max_candidates=16)
        x = torch.empty(nx * ny * ns * nt, dtype=torch.float16, device="cuda")
        nsfrb.generate_noise(x.data_ptr(), "f16", "pst", nx * ny, ns, nt, 900 + k, stream=stream)
        off = delay_table(c.freqs, c.freqs.max(), 134.2, [500.0])[0]
        nsfrb.inject_boxcar(x.data_ptr(), "f16", "pst", nx * ny, ns, nt, pixel=nx * ny - 1, t0=20,
                            width=4, amp=3.0, offsets=off, stream=stream)
        cfgs.append(c)
        cubes.append(x)
    ptrs = [x.data_ptr() for x in cubes]
    print(f"[gpu] batch with {pix} pixel(s) per item", flush=True)
    with nsfrb.Batch(cfgs) as b:
        b.run_separate(ptrs, stream)
        ref = results(b, len(cfgs))
        ref_best = [b.best(i) for i in range(len(cfgs))]
        b.run(ptrs, stream)
        same(results(b, len(cfgs)), ref)
        for i in range(len(cfgs)):
            for g, r in zip(b.best(i), ref_best[i]):
                assert np.array_equal(g, r, equal_nan=True)
    for i, (snr, toa, cands, ntot) in enumerate(ref):     # the pulse sits on each cube's last pixel
        assert ntot >= 1 and cands[0]["x"] + cfgs[i].nx * cands[0]["y"] == cfgs[i].n_pix - 1


def test_injectors_match_their_definition():
    """Batched boxcars and interference added to zero cubes equal the definition
    written out in NumPy (FP32 adds to zero are exact), in both layouts."""
    rng = np.random.default_rng(11)
    n_pix, n_sub, n_t = 37, 16, 90
    for layout in ("tsp", "pst"):
        cubes = [torch.zeros(n_pix * n_sub * n_t, dtype=torch.float32, device="cuda") for _ in range(3)]
        ptrs = [c.data_ptr() for c in cubes]
        boxcars = [(0, 5, 10, 4, 1.5), (2, 5, 80, 16, -2.25), (2, 36, -3, 7, 0.75), (1, 0, 0, 1, 3.0)]
        offsets = rng.integers(0, 9, (len(boxcars), n_sub))
        print(f"[gpu] inject_boxcars layout={layout}", flush=True)
        nsfrb.inject_boxcars(ptrs, "f32", layout, n_pix, n_sub, n_t, boxcars, offsets)
        nsfrb.inject_rfi(ptrs[1], "f32", layout, n_pix, n_sub, n_t, "spike", 33, 1, 0, 0.5)
        nsfrb.inject_rfi(ptrs[1], "f32", layout, n_pix, n_sub, n_t, "stripe", 85, 20, 3, 0.25)
        torch.cuda.synchronize()
        want = np.zeros((3, n_t, n_sub, n_pix), np.float32)            # [cube][t][s][p]
        for (k, p, t0, w, a), off in zip(boxcars, offsets):
            for s in range(n_sub):
                for t in range(t0 + off[s], t0 + off[s] + w):
                    if 0 <= t < n_t:
                        want[k, t, s, p] += np.float32(a)
        want[1, 33, :, :] += np.float32(0.5)
        want[1, 85:, 3, :] += np.float32(0.25)
        for k in range(3):
            got = cubes[k].cpu().numpy()
            got = got.reshape(n_t, n_sub, n_pix) if layout == "tsp" else got.reshape(n_pix, n_sub, n_t).transpose(2, 1, 0)
            assert np.array_equal(got, want[k]), (layout, k)


def test_inject_boxcars_rejects_shared_pixels():
    cube = torch.zeros(4 * 2 * 8, dtype=torch.float32, device="cuda")
    with pytest.raises(nsfrb.NsfrbError):
        nsfrb.inject_boxcars([cube.data_ptr()], "f32", "tsp", 4, 2, 8, [(0, 1, 0, 1, 1.0), (0, 1, 3, 1, 1.0)],
                             np.zeros((2, 2), np.int32))


def test_full_size_batch_graph_equals_separate_and_oracle():
    """The benchmarked batch (64 uneven FP16 cubes, ~108 GB, sides 64-512, 256-4096
    samples): every cube's maps and candidates from the graph replay equal those of
    one plain launch per cube, bit for bit; the smallest cube, copied back from the
    device, is checked against the oracle in full."""
    shapes, total, _ = synth.batch_shapes()
    widths = [1, 2, 4, 8, 16]
    stream = torch.cuda.current_stream().cuda_stream
    cfgs, cubes = [], []
    for k, (side, ns, nt) in enumerate(shapes):
        c = nsfrb.SearchConfig(side, side, nt, np.linspace(1.311, 1.499, ns), C1_DMS, widths, in_dtype="f16",
                               store_dtype="f16", norm="none", layout="pst", snr_threshold=6.0)
        x = torch.empty(side * side * ns * nt, dtype=torch.float16, device="cuda")
        nsfrb.generate_noise(x.data_ptr(), "f16", "pst", side * side, ns, nt, 1000 + k, stream=stream)
        off = delay_table(c.freqs, c.freqs.max(), 134.2, [500.0])[0]
        nsfrb.inject_boxcar(x.data_ptr(), "f16", "pst", side * side, ns, nt, pixel=(side // 2) * side + side // 2,
                            t0=min(20, nt - 8), width=4, amp=1.0, offsets=off, stream=stream)
        cfgs.append(c)
        cubes.append(x)
    ptrs = [x.data_ptr() for x in cubes]
    print(f"[gpu] full-size batch: {len(cfgs)} cubes, {total / 1e9:.1f} GB", flush=True)
    with nsfrb.Batch(cfgs) as b:
        b.run(ptrs, stream)
        got = results(b, len(cfgs))
        assert b.info()["graph"]
        b.run_separate(ptrs, stream)
        same(got, results(b, len(cfgs)))
    k = int(np.argmin([s * s * ns * nt for s, ns, nt in shapes]))
    c = cfgs[k]
    z = cubes[k].cpu().numpy().astype(np.float32).reshape(c.n_pix, c.n_sub, c.n_time)   # [p][s][t]
    o = oracle_run(np.transpose(z, (2, 1, 0)).copy(), c)
    snr, toa, cands, ntot = got[k]
    fin = np.isfinite(o["snr_max"])
    assert np.array_equal(np.isfinite(snr), fin)
    assert np.abs(snr[fin] - o["snr_max"][fin]).max() <= 2e-4
    clear = fin & (o["margin"] > 2e-4)
    np.testing.assert_array_equal(toa[clear], o["toa"][clear])


def test_batch_graph_after_plain_run_with_other_cubes():
    """graph run on cubes A, plain run on cubes B, graph run on B: the last run
    must search B (re-captured), not replay the graph captured for A."""
    rng = np.random.default_rng(21)
    cfgs = uneven_cfgs(rng, 4, "tsp", "f32")
    stream = torch.cuda.current_stream()

    def cubes(seed, pix_shift):
        out = []
        for i, c in enumerate(cfgs):
            cube = synth.noise_cube(c.n_time, c.n_sub, c.n_pix, seed=seed + i)
            off = delay_table(c.freqs, c.freqs.max(), 134.2, [428.0])[0]
            synth.inject_boxcar(cube, (3 + pix_shift) % c.n_pix, 30, off, 8, 4.0)
            out.append(to_device(cube, "f32"))
        return out

    a, bb = cubes(300, 0), cubes(400, 5)
    pa, pb = [x.data_ptr() for x in a], [x.data_ptr() for x in bb]
    with nsfrb.Batch(cfgs) as b:
        print("[gpu] batch graph(A) -> plain(B) -> graph(B)", flush=True)
        b.run_separate(pb, stream.cuda_stream)
        ref_b = results(b, len(cfgs))
        b.run_separate(pa, stream.cuda_stream)
        ref_a = results(b, len(cfgs))
        b.run(pa, stream.cuda_stream)
        assert b.info()["graph"]
        same(results(b, len(cfgs)), ref_a)
        b.use_graph(False)
        b.run(pb, stream.cuda_stream)
        same(results(b, len(cfgs)), ref_b)
        b.use_graph(True)
        b.run(pb, stream.cuda_stream)
        assert b.info()["graph"]
        same(results(b, len(cfgs)), ref_b)
        b.use_graph(False)
        b.run(pa, stream.cuda_stream)
        same(results(b, len(cfgs)), ref_a)
    assert any(not np.array_equal(x[0], y[0]) for x, y in zip(ref_a, ref_b))
