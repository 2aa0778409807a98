"""Seeded synthetic image cubes (input generator shared by tests and benchmark).

This module synthesises inputs only; it holds none of the search's arithmetic.
Cubes are laid out [t][s][p] (time, sub-band, pixel with p = y*nx + x) and
drawn from NumPy's PCG64 generator so that every run with the same seed sees
identical bytes.

Workloads follow the paper's shapes and value distributions: Gaussian image
noise with a per-pixel sigma, boxcar-shaped dispersed pulses (the injection
tests of sections 3.1 and 3.2), broadband zero-DM spikes and narrowband
sub-band stripes (the RFI classes of section 4.3 and appendix B). No survey
data are used; none are available.

Sky model: a pulse of DM `dm` that starts at sample t0 at the reference
(highest) frequency arrives in sub-band s at t0 + round(k*dm*(f_s^-2 -
f_ref^-2)/dt) -- the cold-plasma dispersion law, rounded to whole samples as
the synthetic workload prescribes.
"""
import os

import numpy as np


def noise_cube(nt, ns, npix, seed, sigma_pix=None, dtype=np.float32, block=64):
    """Gaussian noise [t][s][p]; sigma per pixel (default 1).

    Time blocks of `block` samples draw from independent PCG64 streams spawned
    from `seed` (so blocks can be filled by parallel threads; the result does
    not depend on the thread count).
    """
    import concurrent.futures as cf
    cube = np.empty((nt, ns, npix), dtype=np.float32)
    nblk = (nt + block - 1) // block
    seqs = np.random.SeedSequence(seed).spawn(nblk)
    sig = None if sigma_pix is None else np.asarray(sigma_pix, dtype=np.float32)[None, None, :]

    def fill(b):
        rng = np.random.default_rng(seqs[b])
        sl = cube[b * block:(b + 1) * block]
        rng.standard_normal(out=sl, dtype=np.float32)
        if sig is not None:
            np.multiply(sl, sig, out=sl)

    workers = min(16, os.cpu_count() or 1, nblk)
    if workers > 1 and cube.size > (1 << 22):
        with cf.ThreadPoolExecutor(workers) as ex:
            list(ex.map(fill, range(nblk)))
    else:
        for b in range(nblk):
            fill(b)
    return cube.astype(dtype, copy=False)


def arrival_offsets(dm, freqs_ghz, f_ref_ghz, dt_ms, k_dm_ms=4.15):
    """Sky model: per-sub-band arrival offset (samples) of a pulse of this DM."""
    f = np.asarray(freqs_ghz, dtype=np.float64)
    secs = k_dm_ms * float(dm) * (f ** -2.0 - float(f_ref_ghz) ** -2.0)
    return np.rint(secs / float(dt_ms)).astype(np.int64)


def inject_boxcar(cube, p, t0, offsets, width, amp):
    """Add `amp` to samples t0+offsets[s] .. +width-1 of every sub-band at pixel p."""
    nt, ns, _ = cube.shape
    for s in range(ns):
        a = int(t0) + int(offsets[s])
        lo, hi = max(a, 0), min(a + int(width), nt)
        if hi > lo:
            cube[lo:hi, s, p] += np.asarray(amp, dtype=cube.dtype)


def zero_dm_spike(cube, t, amp_pix):
    """Broadband single-sample spike at sample t in every pixel and sub-band."""
    cube[t, :, :] += np.asarray(amp_pix, dtype=cube.dtype)[None, :]


def stripe(cube, s, amp_pix, t_lo=0, t_hi=None):
    """Narrowband stripe: sub-band s raised over [t_lo, t_hi) in every pixel."""
    t_hi = cube.shape[0] if t_hi is None else t_hi
    cube[t_lo:t_hi, s, :] += np.asarray(amp_pix, dtype=cube.dtype)[None, :]


# ---------------------------------------------------------------- configs
C1_FREQS = np.linspace(1.311, 1.499, 4)
C2_FREQS = np.linspace(1.311, 1.499, 16)
DT_MS = 134.2


def widths_pow2(max_pow2, extra=()):
    return [1 << i for i in range(max_pow2.bit_length()) if (1 << i) <= max_pow2] + list(extra)


def config1(seed=0, amp=1.0, t0=20, width=4, dm=500.0, pixel=(16, 16)):
    """Tiny FP32 search: 32x32 px, 4 sub-bands, 64 samples, one injected pulse."""
    nx = ny = 32
    cube = noise_cube(64, 4, nx * ny, seed)
    p = pixel[1] * nx + pixel[0]
    off = arrival_offsets(dm, C1_FREQS, C1_FREQS.max(), DT_MS)
    inject_boxcar(cube, p, t0, off, width, amp)
    meta = dict(nx=nx, ny=ny, freqs=C1_FREQS, f_ref=float(C1_FREQS.max()), dt_ms=DT_MS,
                dms=np.linspace(0.0, 1000.0, 8), widths=[1, 2, 4, 8, 16], theta=6.0,
                injections=[dict(p=p, t0=t0, dm=dm, width=width, amp=amp, offsets=off)])
    return cube, meta


def config2_grid(ns=16, n_dm=32, dm_max=4000.0):
    """The survey search's sub-band centres (GHz), DM trials and widths."""
    return np.linspace(1.311, 1.499, ns), np.linspace(0.0, dm_max, n_dm), widths_pow2(1024, (1200,))


def config2(seed=2, nx=256, ny=256, nt=2048, ns=16, n_pulses=100, n_spikes=20,
            n_stripes=2, rfi_sigma=5.0, n_dm=32, dm_max=4000.0):
    """Survey-shape search: 256x256 px, 16 sub-bands, 2048 samples, pulses and RFI.

    sigma_p ~ U(0.8, 1.2) per pixel; pulses at distinct random pixels with
    DM ~ U(0, dm_max), width = round(exp U(0, ln 1200)), S/N ~ U(6, 50) and
    amplitude S/N * sigma_p / sqrt(width * n_sub); zero-DM spikes of 5 sigma_p
    per sub-band; full-duration sub-band stripes of 5 sigma_p.
    """
    freqs, dms, widths = config2_grid(ns, n_dm, dm_max)
    f_ref = float(freqs.max())
    npix = nx * ny
    rng = np.random.default_rng(seed + 1_000_003)
    sig = rng.uniform(0.8, 1.2, npix).astype(np.float32)
    cube = noise_cube(nt, ns, npix, seed, sig)
    pix = rng.choice(npix, size=n_pulses, replace=False)
    inj = []
    for p in pix:
        dm = rng.uniform(0.0, dm_max)
        w = int(np.rint(np.exp(rng.uniform(0.0, np.log(1200.0)))))
        snr = rng.uniform(6.0, 50.0)
        off = arrival_offsets(dm, freqs, f_ref, DT_MS)
        t_hi = nt - int(off.max()) - w
        t0 = int(rng.integers(0, max(t_hi, 0) + 1))
        amp = snr * float(sig[p]) / np.sqrt(w * ns)
        inject_boxcar(cube, int(p), t0, off, w, amp)
        inj.append(dict(p=int(p), t0=t0, dm=dm, width=w, snr=snr, amp=amp, offsets=off))
    spikes = rng.choice(nt, size=n_spikes, replace=False)
    for t in spikes:
        zero_dm_spike(cube, int(t), rfi_sigma * sig)
    stripes = rng.choice(ns, size=n_stripes, replace=False)
    for s in stripes:
        stripe(cube, int(s), rfi_sigma * sig)
    meta = dict(nx=nx, ny=ny, freqs=freqs, f_ref=f_ref, dt_ms=DT_MS, dms=dms, widths=widths,
                theta=6.0, sigma_pix=sig, injections=inj, spikes=spikes, stripes=stripes)
    return cube, meta


# ------------------------------------------------------ counter-based RNG
PHILOX_M0, PHILOX_M1 = 0xD2511F53, 0xCD9E8D57
PHILOX_W0, PHILOX_W1 = 0x9E3779B9, 0xBB67AE85


def philox4x32_10(counters, key):
    """Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): counters [N,4] uint32, key (k0, k1).

    Each round multiplies words 0 and 2 by the two multipliers (32x32 -> 64
    bits); the new words are (hi(M1*x2) ^ x1 ^ k0, lo(M1*x2), hi(M0*x0) ^ x3 ^ k1,
    lo(M0*x0)); the key is bumped by the Weyl constants between rounds.
    """
    x = np.asarray(counters, dtype=np.uint64).reshape(-1, 4).copy()
    k0, k1 = np.uint64(key[0] & 0xFFFFFFFF), np.uint64(key[1] & 0xFFFFFFFF)
    mask = np.uint64(0xFFFFFFFF)
    for r in range(10):
        if r:
            k0 = (k0 + np.uint64(PHILOX_W0)) & mask
            k1 = (k1 + np.uint64(PHILOX_W1)) & mask
        p0 = np.uint64(PHILOX_M0) * x[:, 0]
        p1 = np.uint64(PHILOX_M1) * x[:, 2]
        n = np.empty_like(x)
        n[:, 0] = (p1 >> np.uint64(32)) ^ x[:, 1] ^ k0
        n[:, 1] = p1 & mask
        n[:, 2] = (p0 >> np.uint64(32)) ^ x[:, 3] ^ k1
        n[:, 3] = p0 & mask
        x = n
    return x.astype(np.uint32)


def philox_blocks(n_blocks, seed):
    """Words of blocks 0..n-1: counter (i, 0, 0, 0), key (seed low, seed high)."""
    i = np.arange(n_blocks, dtype=np.uint64)
    c = np.zeros((n_blocks, 4), dtype=np.uint64)
    c[:, 0] = i & np.uint64(0xFFFFFFFF)
    c[:, 1] = i >> np.uint64(32)
    return philox4x32_10(c, (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)).reshape(-1)


def philox_normals(n, seed, sigma=1.0):
    """Box-Muller normals from Philox blocks, in FP64 (reference for the device generator)."""
    w = philox_blocks((n + 3) // 4, seed).astype(np.float64).reshape(-1, 4)
    u = lambda a: (np.floor(a / 512.0) + 0.5) / 8388608.0
    r0 = np.sqrt(-2.0 * np.log(u(w[:, 0])))
    a0 = 2 * np.pi * u(w[:, 1])
    r1 = np.sqrt(-2.0 * np.log(u(w[:, 2])))
    a1 = 2 * np.pi * u(w[:, 3])
    v = np.stack([r0 * np.cos(a0), r0 * np.sin(a0), r1 * np.cos(a1), r1 * np.sin(a1)], axis=1).reshape(-1)
    return sigma * v[:n]


# ------------------------------------------------------------ simulated PSF
def snapshot_psf(half=24, seed=11, n_ew=40, n_ns=16, lobe_px=0.6):
    """Snapshot dirty beam of a T-shaped array (an east-west arm and a
    north-south arm, as the DSA-110), on a (2 half + 1)^2 pixel grid centred on
    the middle pixel: B(l, m) = sum over antenna pairs a != b of
    cos(2 pi (u_ab l + v_ab m)) / (N (N - 1)), peak 1 at the centre, with
    positive and negative sidelobes. Antennas sit at jittered, roughly even
    spacings; the pixel scale puts the main lobe's half width near lobe_px."""
    rng = np.random.default_rng(seed)
    ew = np.sort(rng.uniform(-1.0, 1.0, n_ew))
    ns = np.sort(rng.uniform(0.05, 1.0, n_ns))
    x = np.concatenate([ew, np.zeros(n_ns)])
    y = np.concatenate([np.zeros(n_ew), ns])
    scale = 0.5 / (lobe_px * (x.max() - x.min()))          # cycles per pixel per unit baseline
    g = np.arange(-half, half + 1) * scale
    ph_x = np.exp(2j * np.pi * np.outer(x, g))              # [antenna][l]
    ph_y = np.exp(2j * np.pi * np.outer(y, g))              # [antenna][m]
    v = np.einsum("al,am->ml", ph_x, ph_y)                  # voltage sum [m][l]
    n = x.size
    beam = (np.abs(v) ** 2 - n) / (n * (n - 1))
    return (beam / beam[half, half]).astype(np.float32)


def batch_shapes(seed=4, n=64, cap_bytes=128e9):
    """Cube shapes (side, sub-bands, samples) of the batched workload: side
    log-uniform 64-512, samples log-uniform 256-4096, sub-bands 8 or 16; redrawn
    with seed + 1 until the FP16 total fits the cap. Returns (shapes, bytes, seed)."""
    while True:
        rng = np.random.default_rng(seed)
        side = np.rint(np.exp(rng.uniform(np.log(64), np.log(512), n))).astype(int)
        nt = np.rint(np.exp(rng.uniform(np.log(256), np.log(4096), n))).astype(int)
        ns = rng.choice([8, 16], n)
        total = float(np.sum(side * side * ns * nt * 2))
        if total <= cap_bytes:
            return [(int(a), int(b), int(c)) for a, b, c in zip(side, ns, nt)], total, seed
        seed += 1
