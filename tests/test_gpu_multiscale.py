"""GPU parity of the multi-timescale search (needs an MI355X).

The raw cube is binned by 5 and 75 samples and each timescale is searched
(native DMs; 5x the DMs on the 5x-binned data; DM 0 alone on the 75x-binned
data), as in section 2.2 of the paper. Checked against the oracle:
  * binning: bit-exact for FP32, FP16 and BF16 input;
  * per timescale: the rules of tests/test_gpu_search.py (delay table, noise
    statistics and normalised cube bit-exact; S/N within 1e-4; indices exact
    where the oracle's margins exceed 2e-4);
  * merged candidates: S/N order across timescales, identities where unambiguous.
"""
import numpy as np
import pytest

from oracle import search as osr
from paper_2510_18136_amd import nsfrb, synth
from tests._lib import ensure_built
from tests.test_gpu_search import EPS, TOL, compare, dw_margin, input_values, to_device

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FACTORS, DM_SCALES = (1, 5, 75), (1.0, 5.0, 0.0)


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_built()
    assert torch.cuda.is_available()


def gpu_view(s, cfg):
    cands, ntot, st = s.candidates()
    bs, bd, bw, bt = s.best()
    snr, toa = s.maps()
    out = dict(cands=cands, n_total=ntot, status=st, snr=snr, toa=toa, best=bs, best_d=bd, best_w=bw, best_t=bt,
               delays=s.delay_table(), flags=s.flag_count(), z=s.zcube()[0])
    out["med"], out["sig"] = s.noise_stats()
    return out


def oracle_scale(xb, cfg):
    r = osr.search(xb, cfg.freqs, float(cfg.c.f_ref_ghz), cfg.c.dt_ms, cfg.dms, list(cfg.widths), cfg.nx,
                   norm=cfg.norm, store=cfg.store_dtype, theta=float(cfg.c.snr_threshold),
                   k_max=cfg.max_candidates)
    sm, toa, margin = osr.snr_toa_margin_maps(r["z"], r["delays"], list(cfg.widths))
    r["margin"] = margin
    return r


def make_cube(seed, nt, ns, npix):
    rng = np.random.default_rng(seed)
    cube = rng.standard_normal((nt, ns, npix)).astype(np.float32)
    freqs = np.linspace(1.311, 1.499, ns)
    for k, (w, amp, dm) in enumerate([(3, 3.0, 400.0), (40, 1.2, 1500.0), (300, 0.5, 0.0), (150, 0.8, 2500.0)]):
        off = synth.arrival_offsets(dm, freqs, freqs.max(), synth.DT_MS)
        synth.inject_boxcar(cube, 3 + 7 * k, int(rng.integers(0, nt - off.max() - w)), off, w, amp)
    return cube, freqs


@pytest.mark.parametrize("in_dtype", ["f32", "f16", "bf16"])
def test_bin_time_bit_exact(in_dtype):
    rng = np.random.default_rng(5)
    x = (rng.standard_normal((157, 3, 50)) * 3).astype(np.float32)
    xd = to_device(x, in_dtype)
    vals = input_values(x, in_dtype)
    for f in (1, 5, 75, 157):
        out = torch.zeros((157 // f, 3, 50), dtype=torch.float32, device="cuda")
        print(f"[gpu] bin_time dtype={in_dtype} factor={f}", flush=True)
        nsfrb.bin_time(xd.data_ptr(), in_dtype, 157, 3, 50, f, out.data_ptr(),
                       torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy(), osr.bin_time(vals, f))


@pytest.mark.parametrize("store,nt,in_dtype", [("f32", 600, "f32"), ("f16", 751, "f32"), ("bf16", 375, "f32"),
                                               ("f32", 1210, "f16"), ("f16", 908, "bf16")])
def test_multiscale_matches_oracle(store, nt, in_dtype):
    """1210 and 908 samples leave 2 and 1 trailing 5-sample bins past the last
    whole 75-sample bin, so the one-read binning of both factors has a partial
    last group."""
    nx, ny, ns = 16, 8, 8
    cube, freqs = make_cube(31 + nt, nt, ns, nx * ny)
    cfg = nsfrb.SearchConfig(nx, ny, nt, freqs, np.linspace(0, 1000, 6), [1, 2, 4, 8, 16], store_dtype=store,
                             in_dtype=in_dtype, snr_threshold=4.0, max_candidates=25)
    xd = to_device(cube, in_dtype)
    with nsfrb.MultiScale(cfg, FACTORS, DM_SCALES) as ms:
        print(f"[gpu] multiscale store={store} nt={nt} in={in_dtype}", flush=True)
        ms.run(xd.data_ptr(), torch.cuda.current_stream().cuda_stream)
        merged, mtot, mst = ms.candidates()
        views = [gpu_view(ms.scale(i), ms.cfgs[i]) for i in range(len(FACTORS))]
        cfgs = ms.cfgs
    torch.cuda.synchronize()
    orc = []
    for f, c, g in zip(FACTORS, cfgs, views):
        vals = input_values(cube, in_dtype)
        xb = vals if f == 1 else osr.bin_time(vals, f)
        o = oracle_scale(xb, c)
        compare(g, o, c, tol=TOL if store == "f32" else 2e-4)
        orc.append(o)
    theta = float(cfg.c.snr_threshold)
    near = any((np.isfinite(o["best"]) & (np.abs(o["best"] - theta) <= EPS)).any() for o in orc)
    if not near:
        assert mtot == sum(o["n_total"] for o in orc)
    ref = sorted([(-c["snr"], i, c["y"] * nx + c["x"], c) for i, o in enumerate(orc) for c in o["candidates"]],
                 key=lambda r: r[:3])[:cfg.max_candidates]
    assert len(merged) == len(ref)
    tol = TOL if store == "f32" else 2e-4
    for k, (g, r) in enumerate(zip(merged, ref)):
        assert abs(g["snr"] - r[3]["snr"]) <= tol
        gaps = [abs(r[3]["snr"] - q[3]["snr"]) for j, q in enumerate(ref) if j != k]
        if min(gaps, default=np.inf) > EPS:
            assert (g["scale"], g["x"], g["y"]) == (r[1], r[3]["x"], r[3]["y"])


def test_survey_shape_sampled_parity():
    """The three timescales at the survey shape (256x256 px, 16 sub-bands, 2048
    samples; 32 DMs 0-4000 native, the same 32 times 5 on the 5x-binned cube, DM 0
    on the 75x-binned one; widths 1-16 at each), FP32: at every injected pulse's
    pixel and 60 random ones, each timescale's statistics are bit-exact and its
    S/N maps and best trials within 1e-4 of the oracle's search of the binned
    samples, with unique TOAs and trial indices exact; the merged candidate list
    is the S/N-ordered head of the GPU's own per-timescale best maps."""
    cube, meta = synth.config2(seed=2)
    cfg = nsfrb.SearchConfig(meta["nx"], meta["ny"], cube.shape[0], meta["freqs"], meta["dms"], [1, 2, 4, 8, 16],
                             snr_threshold=meta["theta"], max_candidates=10)
    x = torch.from_numpy(cube).cuda()
    with nsfrb.MultiScale(cfg, FACTORS, DM_SCALES) as ms:
        print("[gpu] multiscale survey shape", flush=True)
        ms.run(x.data_ptr(), torch.cuda.current_stream().cuda_stream)
        merged, mtot, _ = ms.candidates()
        views = []
        for i in range(len(FACTORS)):
            v = ms.scale(i)
            views.append((v.maps(), v.best(), v.noise_stats()))
        cfgs = ms.cfgs
    del x
    rng = np.random.default_rng(13)
    pix = np.unique(np.concatenate([[j["p"] for j in meta["injections"]], rng.choice(cfg.n_pix, 60, replace=False)]))
    sub = np.ascontiguousarray(cube[:, :, pix])
    theta = meta["theta"]
    ref = []
    for i, (f, c, ((snr, toa), (bs, bd, bw, _), (med, sig))) in enumerate(zip(FACTORS, cfgs, views)):
        xb = sub if f == 1 else osr.bin_time(sub, f)
        assert xb.shape[0] == c.n_time
        o = osr.search(xb, c.freqs, float(c.c.f_ref_ghz), c.c.dt_ms, c.dms, list(c.widths), len(pix), theta=theta,
                       k_max=10)
        _, _, margin = osr.snr_toa_margin_maps(o["z"], o["delays"], list(c.widths))
        np.testing.assert_array_equal(med[pix], o["med"])
        np.testing.assert_array_equal(sig[pix], o["sigma"])
        g = snr[:, :, pix]
        fin = np.isfinite(o["snr_max"])
        assert np.array_equal(np.isfinite(g), fin)
        assert np.abs(g[fin] - o["snr_max"][fin]).max() <= TOL
        clear = fin & (margin > EPS)
        np.testing.assert_array_equal(toa[:, :, pix][clear], o["toa"][clear])
        assert np.abs(bs[pix] - o["best"]).max() <= TOL
        ok = dw_margin(o["snr_max"]) > EPS
        np.testing.assert_array_equal(bd[pix][ok], o["best_d"][ok])
        np.testing.assert_array_equal(bw[pix][ok], o["best_w"][ok])
        ref += [(-float(bs[p]), i, int(p)) for p in np.flatnonzero(bs >= theta)]
    ref.sort()
    assert mtot == len(ref)
    assert [(g["scale"], g["y"] * cfg.nx + g["x"]) for g in merged] == [(i, p) for _, i, p in ref[:10]]
    assert all(g["snr"] == -s for g, (s, _, _) in zip(merged, ref))
