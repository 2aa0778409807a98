"""Training and evaluation of the candidate classifier on cutouts the search makes.

Section 2.3 of the paper runs a CNN over the image cube centred on each
candidate's TOA (position, time, frequency); its sigmoid output is the RFI
probability p_rfi, it is trained with Adam on a binary cross-entropy loss, and
section 3.2 keeps candidates with p_rfi below a threshold (15% nominal, 50%
looser). This module builds that loop on the GPU, with every step in the
library's kernels:

  device noise (Philox4x32-10 + Box-Muller)  ->  injected pulses, sidelobe
  ghosts and RFI  ->  batched search (FP64 median/MAD, FP16 z, de-dispersion,
  boxcars, S/N, per-pixel best trial)  ->  dedispersion-aligned cutouts of the
  requested pixels  ->  BF16 MFMA forward/backward + Adam.

Cubes: 64 x 64 pixels, 16 sub-bands evenly spanning 1.311-1.499 GHz, 256
samples of 134.2 ms, N(0, 1) noise. Search grid: 8 DMs evenly spanning 0-1000
pc cm^-3, widths {1, 2, 4, 8, 16} (the small-survey grid). Each cube is one of
  * sky: four dispersed boxcar pulses, S/N U(5, 50), DM U(0, 1000), width
    log-uniform 1-16 samples, amplitude S/N / sqrt(16 w), at pixels at least
    17 apart in x or y (no cutout holds two unrelated pulses: transients are
    sparse on the sky); each pulse has, with probability 1/2, one or two
    sidelobe ghosts: copies at 0.1-0.3x amplitude 3-12 pixels away;
  * spike: one to three zero-DM spikes over all pixels (one sample, every
    sub-band, 1.5-10 sigma per sub-band);
  * stripe: one to three narrowband stripes over all pixels (one sub-band,
    8-96 samples, 3-15 sigma).
A candidate is the search's best (DM, width, TOA) trial at a pixel. Labels
follow p_rfi: 0 = astrophysical (pulse pixels), 1 = RFI or noise (ghost
pixels, the two highest-S/N pixels of a sky cube away from every injection
plus one random such pixel, and eight random pixels of every RFI cube).

Training is one pass over freshly generated cutouts (batch 64, Adam, the
learning rate following a cosine from lr to lr/100). The generator is
counter-based: round r of cubes draws from a NumPy generator seeded with
(seed, r), so a run checkpointed after round r (weights, Adam state and step
count through the library's checkpoint, the round counter in its user word,
the cutout and step counts beside it) resumes with the result it would have
had without the stop.

The plain S/N >= 6 threshold is the baseline and the fallback: evaluate()
reports its recall and false candidates next to the classifier's. The
classifier's operating point (keep p_rfi < cut) is chosen on a validation
split: the smallest cut whose validation recall reaches the threshold's
validation recall plus two binomial standard errors, so that the held-out
recall is not below the threshold's by sampling noise alone (one standard
error left the seeded 200k run's held-out recall 0.14 points below the
threshold's).

Usage: python -m paper_2510_18136_amd.train_classifier --train 200000 \
           --val 10000 --heldout 10000 --out <dir>
"""
import argparse
import json
import math
import os
import time

import numpy as np

from . import nsfrb

FREQS = np.linspace(1.311, 1.499, 16)
DMS = np.linspace(0.0, 1000.0, 8)
WIDTHS = np.array([1, 2, 4, 8, 16], np.int32)
NX = NY = 64
NT = 256
N_SUB = 16
CUT_T = 64
SNR_THRESHOLD = 6.0
KINDS = ("pulse", "ghost", "noise", "spike", "stripe")
RECALL_MARGIN_SE = 2.0      # operating point: threshold's validation recall + this many binomial SEs


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the classifier pipeline needs a GPU (HIP device)")
    return torch


def pulse_offsets(dm):
    """Per-sub-band sample shifts of a pulse of true DM `dm` (the search's delay law)."""
    return nsfrb.SearchConfig(NX, NY, NT, FREQS, [dm], WIDTHS).delays()[0]


def plan_cube(rng, k, kind):
    """Host-side plan of cube k: boxcars (cube, pixel, t0, width, amp) with their
    sub-band offsets, interference events (kind, t0, len, sub-band, amp) and the
    injected pixels to cut out ((x, y), label kind, S/N of the injection)."""
    plan = dict(kind=kind, boxcars=[], offsets=[], rfi=[], req=[], occupied=[])
    if kind == "sky":
        taken = set()
        mains = []
        n_pulse = tries = 0
        while n_pulse < 4 and tries < 10000:
            tries += 1
            x, y = int(rng.integers(0, NX)), int(rng.integers(0, NY))
            if any(max(abs(x - a), abs(y - b)) < 17 for a, b in plan["occupied"]):
                continue
            mains.append((x, y))
            snr = rng.uniform(5.0, 50.0)
            w = int(round(math.exp(rng.uniform(0.0, math.log(16.0)))))
            dm = rng.uniform(0.0, 1000.0)
            t0 = int(rng.integers(40, NT - 40 - w))
            amp = snr / math.sqrt(N_SUB * w)
            off = pulse_offsets(dm)
            plan["boxcars"].append((k, y * NX + x, t0, w, amp))
            plan["offsets"].append(off)
            plan["occupied"].append((x, y))
            taken.add((x, y))
            plan["req"].append(((x, y), "pulse", snr))
            n_pulse += 1
            if rng.random() < 0.5:
                for _ in range(int(rng.integers(1, 3))):
                    for _try in range(20):
                        r = int(rng.integers(3, 13))
                        dx, dy = int(rng.integers(-r, r + 1)), int(rng.integers(-r, r + 1))
                        if max(abs(dx), abs(dy)) != r:
                            continue
                        gx, gy = x + dx, y + dy
                        if not (0 <= gx < NX and 0 <= gy < NY) or (gx, gy) in taken:
                            continue
                        if any(max(abs(gx - a), abs(gy - b)) < 17 for a, b in mains[:-1]):
                            continue                  # a ghost's cutout holds only its own source
                        frac = rng.uniform(0.1, 0.3)
                        plan["boxcars"].append((k, gy * NX + gx, t0, w, amp * frac))
                        plan["offsets"].append(off)
                        taken.add((gx, gy))
                        plan["occupied"].append((gx, gy))
                        plan["req"].append(((gx, gy), "ghost", snr * frac))
                        break
    else:
        for _ in range(int(rng.integers(1, 4))):
            if kind == "spike":
                plan["rfi"].append(("spike", int(rng.integers(8, NT - 8)), 1, 0, float(rng.uniform(1.5, 10.0))))
            else:
                ln = int(rng.integers(8, 97))
                plan["rfi"].append(("stripe", int(rng.integers(0, NT - ln)), ln, int(rng.integers(0, N_SUB)),
                                    float(rng.uniform(3.0, 15.0))))
    return plan


def candidate_records(rng, k, plan, snr, dmi, toa):
    """Candidates of cube k from the search's per-pixel best arrays: records
    (cube, px, py, dm_index, toa, label, snr, kind), label 0 = astrophysical."""
    recs = []
    if plan["kind"] == "sky":
        for (x, y), kind, _ in plan["req"]:
            p = y * NX + x
            recs.append((k, x, y, int(dmi[p]), int(toa[p]), 0 if kind == "pulse" else 1, float(snr[p]), kind))
        ys, xs = np.divmod(np.arange(NX * NY), NX)
        far = np.ones(NX * NY, bool)
        for a, b in plan["occupied"]:
            far &= np.maximum(np.abs(xs - a), np.abs(ys - b)) > 3
        cand = np.flatnonzero(far)
        top = cand[np.argsort(-snr[cand], kind="stable")[:2]]
        for p in list(top) + [int(rng.choice(cand))]:
            recs.append((k, int(xs[p]), int(ys[p]), int(dmi[p]), int(toa[p]), 1, float(snr[p]), "noise"))
    else:
        for p in rng.choice(NX * NY, size=8, replace=False):
            y, x = divmod(int(p), NX)
            recs.append((k, x, y, int(dmi[p]), int(toa[p]), 1, float(snr[p]), plan["kind"]))
    return recs


class CutoutSource:
    """Labelled candidate cutouts generated and searched on the GPU."""

    def __init__(self, seed, n_cubes=16, device=0, first_round=0):
        torch = _torch()
        self.torch = torch
        self.seed = seed
        self.rounds = first_round           # rounds generated so far (the generator's counter)
        self.n_cubes = n_cubes
        self.cfg = nsfrb.SearchConfig(NX, NY, NT, FREQS, DMS, WIDTHS, in_dtype="f32", store_dtype="f16",
                                      norm="pixel_subband", snr_threshold=0.0, max_candidates=16, device=device)
        self.batch = nsfrb.Batch([self.cfg] * n_cubes)
        self.delays = self.cfg.delays()                             # [n_dm][n_sub] search delay table
        self.raw = torch.empty((n_cubes, NX * NY * N_SUB * NT), dtype=torch.float32, device=f"cuda:{device}")

    def round(self):
        """Generate and search n_cubes cubes; returns (z pointers, candidate records)."""
        rng, torch = np.random.default_rng([self.seed, self.rounds]), self.torch
        self.rounds += 1
        kinds = rng.choice(["sky", "spike", "stripe"], size=self.n_cubes, p=[0.6, 0.2, 0.2])
        ptrs = [int(self.raw[k].data_ptr()) for k in range(self.n_cubes)]
        plans = [plan_cube(rng, k, str(kinds[k])) for k in range(self.n_cubes)]
        for k in range(self.n_cubes):
            nsfrb.generate_noise(ptrs[k], "f32", "tsp", NX * NY, N_SUB, NT, int(rng.integers(1, 2 ** 63)))
            for kind, t0, ln, sb, amp in plans[k]["rfi"]:
                nsfrb.inject_rfi(ptrs[k], "f32", "tsp", NX * NY, N_SUB, NT, kind, t0, ln, sb, amp)
        boxcars = [b for pl in plans for b in pl["boxcars"]]
        if boxcars:
            offsets = np.stack([o for pl in plans for o in pl["offsets"]])
            nsfrb.inject_boxcars(ptrs, "f32", "tsp", NX * NY, N_SUB, NT, boxcars, offsets)
        torch.cuda.synchronize()
        self.batch.run(ptrs)
        records, zptrs = [], []
        for k in range(self.n_cubes):
            snr, dmi, _, toa = self.batch.best(k)
            zptrs.append(self.batch.zcube_device(k))
            records += candidate_records(rng, k, plans[k], snr, dmi, toa)
        return zptrs, records

    def close(self):
        self.batch.close()


def _extract(clf, src, zptrs, recs, out):
    clf.cutouts(zptrs, "f16", NX, NY, N_SUB, NT, src.delays, [r[:5] for r in recs], out.data_ptr())


def train(clf, n_train, seed, lr=1e-3, batch=64, n_cubes=16, log=print, ckpt=None, resume=False,
          stop_after_rounds=None):
    """One pass over n_train fresh cutouts. With `ckpt` (a path), a checkpoint is
    written after every round of cubes (ckpt, plus ckpt + '.json' with the
    cutout and step counts); resume=True continues from it. stop_after_rounds
    ends the run early after that many rounds (a stopped job, for tests)."""
    torch = _torch()
    seen, steps, losses, first_round = 0, 0, [], 0
    if resume:
        first_round = clf.load(ckpt)
        with open(ckpt + ".json") as f:
            meta = json.load(f)
        seen, steps, losses = meta["seen"], meta["steps"], [tuple(x) for x in meta["losses"]]
        assert meta["rounds"] == first_round
    src = CutoutSource(seed, n_cubes, first_round=first_round)
    xbuf = torch.empty((batch, CUT_T, 32, 32, N_SUB), dtype=torch.int16, device="cuda")
    ybuf = torch.empty(batch, dtype=torch.float32, device="cuda")
    t_gen = t_step = 0.0
    t_start = time.time()
    while seen < n_train:
        if stop_after_rounds is not None and src.rounds >= stop_after_rounds:
            break
        t0 = time.time()
        r = src.rounds
        zptrs, recs = src.round()
        t_gen += time.time() - t0
        order = np.random.default_rng([seed + 17, r]).permutation(len(recs))
        for i in range(0, len(order), batch):
            if seen >= n_train:
                break
            sel = [recs[j] for j in order[i:i + batch]][: n_train - seen]
            t1 = time.time()
            clf.set_lr(lr * (0.01 + 0.99 * 0.5 * (1.0 + math.cos(math.pi * seen / n_train))))
            _extract(clf, src, zptrs, sel, xbuf)
            ybuf[: len(sel)].copy_(torch.tensor([r[5] for r in sel], dtype=torch.float32))
            want = steps % 50 == 0
            loss = clf.train_step(xbuf.data_ptr(), ybuf.data_ptr(), len(sel), update=True, want_loss=want)
            if want:
                losses.append((seen, float(loss)))
                log(f"[train] cutouts {seen:7d}  loss {loss:.4f}  elapsed {time.time() - t_start:.1f}s")
            t_step += time.time() - t1
            seen += len(sel)
            steps += 1
        if ckpt:
            torch.cuda.synchronize()
            clf.save(ckpt, user_counter=src.rounds)
            with open(ckpt + ".json", "w") as f:
                json.dump(dict(rounds=src.rounds, seen=seen, steps=steps, losses=losses), f)
    torch.cuda.synchronize()
    src.close()
    return dict(cutouts=seen, steps=steps, seconds=time.time() - t_start, search_gen_seconds=t_gen,
                extract_train_seconds=t_step, loss_curve=losses)


def score(clf, n, seed, batch=64, n_cubes=16):
    """p_rfi, S/N, labels and kinds of n fresh cutouts."""
    torch = _torch()
    src = CutoutSource(seed, n_cubes)
    xbuf = torch.empty((batch, CUT_T, 32, 32, N_SUB), dtype=torch.int16, device="cuda")
    pbuf = torch.empty(batch, dtype=torch.float32, device="cuda")
    probs, snrs, labels, kinds = [], [], [], []
    while len(probs) < n:
        zptrs, recs = src.round()
        for i in range(0, len(recs), batch):
            sel = recs[i:i + batch][: n - len(probs)]
            if not sel:
                break
            _extract(clf, src, zptrs, sel, xbuf)
            clf.infer(xbuf.data_ptr(), len(sel), pbuf.data_ptr())
            torch.cuda.synchronize()
            probs += pbuf[: len(sel)].cpu().tolist()
            snrs += [r[6] for r in sel]
            labels += [r[5] for r in sel]
            kinds += [r[7] for r in sel]
    src.close()
    return np.array(probs), np.array(snrs), np.array(labels), np.array(kinds)


def operating_point(p, label, target_recall):
    """Smallest p_rfi cut (keep p < cut) whose recall on label-0 cutouts reaches target_recall."""
    pos = np.sort(p[label == 0])
    if pos.size == 0:
        return 0.5
    k = int(math.ceil(target_recall * pos.size))
    k = min(max(k, 1), pos.size)
    return float(np.nextafter(pos[k - 1], np.inf))


def summarise(keep, label, kinds):
    pos = label == 0
    out = dict(recall=float(keep[pos].mean()) if pos.any() else None,
               detected=int(keep[pos].sum()), false_candidates=int(keep[~pos].sum()))
    out["false_by_kind"] = {k: int((keep & (kinds == k)).sum()) for k in KINDS if k != "pulse"}
    return out


def evaluate(val, held):
    """Threshold vs classifier on held-out cutouts; operating point from the validation split."""
    pv, sv, lv, _ = val
    ph, sh, lh, kh = held
    thr_val_recall = float((sv[lv == 0] >= SNR_THRESHOLD).mean())
    n_pos = int((lv == 0).sum())
    target = min(1.0, thr_val_recall + RECALL_MARGIN_SE * math.sqrt(thr_val_recall * (1.0 - thr_val_recall)
                                                                   / max(n_pos, 1)))
    cut = operating_point(pv, lv, target)
    res = dict(n=int(lh.size), n_astrophysical=int((lh == 0).sum()), n_rfi_or_noise=int((lh == 1).sum()),
               n_by_kind={k: int((kh == k).sum()) for k in KINDS})
    res["snr_threshold"] = dict(theta=SNR_THRESHOLD, **summarise(sh >= SNR_THRESHOLD, lh, kh))
    res["classifier_matched"] = dict(p_rfi_below=cut, validation_threshold_recall=thr_val_recall,
                                     validation_target_recall=target,
                                     **summarise(ph < cut, lh, kh))
    for c in (0.15, 0.5):
        res[f"classifier_p{int(c * 100)}"] = dict(p_rfi_below=c, **summarise(ph < c, lh, kh))
    res["snr_and_classifier_p50"] = dict(**summarise((sh >= SNR_THRESHOLD) & (ph < 0.5), lh, kh))
    thr_false = res["snr_threshold"]["false_candidates"]
    clf_false = res["classifier_matched"]["false_candidates"]
    res["false_candidate_reduction"] = (thr_false / clf_false) if clf_false else float("inf")
    return res


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--train", type=int, default=200000)
    ap.add_argument("--val", type=int, default=10000)
    ap.add_argument("--heldout", type=int, default=10000)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--out", default="classifier_run")
    ap.add_argument("--resume", action="store_true", help="continue from <out>/checkpoint.bin")
    a = ap.parse_args(argv)
    _torch()                     # torch's HIP runtime first, then the library (one runtime per process)
    os.makedirs(a.out, exist_ok=True)
    with nsfrb.Classifier(max_batch=a.batch, n_time=CUT_T, ny=32, lr=a.lr, seed=a.seed) as clf:
        tr = train(clf, a.train, seed=a.seed * 1000 + 1, lr=a.lr, batch=a.batch, log=lambda m: print(m, flush=True),
                   ckpt=os.path.join(a.out, "checkpoint.bin"), resume=a.resume)
        np.save(os.path.join(a.out, "params.npy"), clf.params())
        print(f"[train] done: {tr['cutouts']} cutouts in {tr['seconds']:.1f}s", flush=True)
        val = score(clf, a.val, seed=a.seed * 1000 + 2, batch=a.batch)
        held = score(clf, a.heldout, seed=a.seed * 1000 + 3, batch=a.batch)
    res = dict(train={k: v for k, v in tr.items()}, lr=a.lr, batch=a.batch, evaluation=evaluate(val, held))
    with open(os.path.join(a.out, "report.json"), "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res["evaluation"], indent=1), flush=True)


if __name__ == "__main__":
    main()
