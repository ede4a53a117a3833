"""Learned specialization picker (cost model) and its evaluation.

The exhaustive autotuner compiles and times every candidate specialization
C(s) of a shape s; the picker instead predicts each candidate's run time with
a small MLP and compiles only the predicted best.  The network (features ->
64 -> 64 -> 1, ReLU, FP32) is trained on GPU with the library's own kernels
(SJ_MLP_BWD for the loss gradient, SJ_ADAM for the update, SJ_MLP_FWD for
prediction), on timings the library itself gathers with sj_time_run.  This is
the profile-guided, adaptive specialization named as future work in ClangJIT
section 6.

Shapes (LTimes): Z = k^3 with k ~ U{8..64}, G ~ U{8..128}, D = 8 U{2..32},
NM ~ U{4, 9, 16, 36, 64}, dtype ~ U{FP64, BF16x3}.  Candidates:
  FP64, column axis innermost (DGZ, DZG, GDZ, ZDG): DIRECT, tile_n in {1, 2},
      order in {ascending, rotated}, unroll 8, block 256; FP64-MFMA columns
      with default tiles, order in {ascending, rotated};
  FP64, D innermost (GZD, ZGD): FP64-MFMA rows, tile_n in {1, 2, 4};
  BF16x3 (column layouts only): columns per lane in {1, 4} (4 when it
      divides the contiguous extent), block 256.
The cost of a candidate is the median of 3 timed launches of one LTimes (after
one warm-up), with L2 and the last-level cache flushed first when the working
set is under 512 MB.  Regret of a pick: t(pick) / min_c t(c) - 1.
"""
from __future__ import annotations

import json
import math
import time

import numpy as np

from . import sj

LAYOUTS = sj.LAYOUTS
COLUMN_LAYOUTS = ("DGZ", "DZG", "GDZ", "ZDG")
NFEAT = 24
WIDTH = 64


def sample_shape(rng: np.random.Generator) -> dict:
    k = int(rng.integers(8, 65))
    return dict(Z=k ** 3, G=int(rng.integers(8, 129)), D=8 * int(rng.integers(2, 33)),
                NM=int(rng.choice([4, 9, 16, 36, 64])),
                dtype=int(rng.choice([sj.SJ_F64, sj.SJ_BF16X3])))


def contiguous_extent(layout: str, Z: int, G: int) -> int:
    return {"DGZ": G * Z, "DZG": G * Z, "GDZ": Z, "ZDG": G}.get(layout, 1)


def candidates(shape: dict) -> list:
    out = []
    if shape["dtype"] == sj.SJ_F64:
        for lay in LAYOUTS:
            if lay in COLUMN_LAYOUTS:
                ext = contiguous_extent(lay, shape["Z"], shape["G"])
                for vec in (1, 2):
                    if ext % vec:
                        continue
                    for order in (1, 2):
                        out.append(dict(layout=lay, variant=sj.SJ_VAR_DIRECT, tile_n=vec, unroll=8, block=256,
                                        order=order))
                for order in (1, 2):
                    out.append(dict(layout=lay, variant=sj.SJ_VAR_MFMA, order=order))
            else:
                for rt in (1, 2, 4):
                    out.append(dict(layout=lay, variant=sj.SJ_VAR_MFMA, tile_n=rt, block=256))
    else:
        for lay in COLUMN_LAYOUTS:
            ext = contiguous_extent(lay, shape["Z"], shape["G"])
            for cpl in (1, 4):
                if ext % cpl == 0:
                    out.append(dict(layout=lay, variant=sj.SJ_VAR_MFMA, tile_n=cpl, block=256))
    return out


def default_candidate(shape: dict) -> dict:
    """What a caller gets without tuning: Kripke's default nesting DGZ with the
    library's default tile parameters."""
    return dict(layout="DGZ")


def features(shape: dict, cand: dict) -> np.ndarray:
    """Raw (unnormalized) feature vector of NFEAT floats."""
    f = np.zeros(NFEAT, dtype=np.float64)
    Z, G, D, NM = shape["Z"], shape["G"], shape["D"], shape["NM"]
    lay = cand.get("layout", "DGZ")
    esz = 8 if shape["dtype"] == sj.SJ_F64 else 4
    f[0:4] = [math.log2(Z), math.log2(G), math.log2(D), math.log2(NM)]
    f[4] = 1.0 if shape["dtype"] == sj.SJ_F64 else 0.0
    f[5] = 1.0 - f[4]
    f[6 + LAYOUTS.index(lay)] = 1.0
    var = cand.get("variant", 0)
    if var == 0:
        var = sj.SJ_VAR_MFMA if (shape["dtype"] != sj.SJ_F64 or lay not in COLUMN_LAYOUTS) else sj.SJ_VAR_DIRECT
    f[12 + (var - 1)] = 1.0
    f[15] = math.log2(max(1, cand.get("tile_n", 0) or 1))
    f[16] = cand.get("unroll", 8) / 16.0
    f[17] = cand.get("block", 256) / 512.0
    f[18] = 1.0 if cand.get("order", 0) == 2 else 0.0
    ext = contiguous_extent(lay, Z, G)
    f[19] = math.log2(ext * esz)                          # contiguous run in bytes
    f[20] = math.log2((D + NM) * G * Z * esz)             # algorithmic bytes
    f[21] = math.log2(2.0 * D * NM * G * Z)               # flops
    f[22] = math.log2(max(1, ext) * esz * 1.0) if lay in ("DGZ", "DZG") else math.log2(Z * esz)  # row stride proxy
    f[23] = 1.0
    return f


# ------------------------------------------------------------------ timing

class Buffers:
    """Device buffers large enough for every sampled shape, allocated once;
    a shape uses their prefixes.  Values come from the counter generator."""

    def __init__(self, max_elems_psi: int, max_elems_phi: int, max_l: int):
        import torch

        from sj_inputs import device as gdev
        import sj_inputs as gen
        self.psi64 = torch.empty(max_elems_psi, dtype=torch.float64, device="cuda")
        self.phi64 = torch.empty(max_elems_phi, dtype=torch.float64, device="cuda")
        self.psi32 = torch.empty(max_elems_psi, dtype=torch.float32, device="cuda")
        self.phi32 = torch.empty(max_elems_phi, dtype=torch.float32, device="cuda")
        self.L = torch.empty(max_l, dtype=torch.float64, device="cuda")
        gdev.fill(self.psi64, 1, gen.ARR_PSI, gdev.DIST_U01)
        gdev.fill(self.psi32, 1, gen.ARR_PSI, gdev.DIST_U01_24)
        gdev.fill(self.L, 1, gen.ARR_L, gdev.DIST_SYM)
        self.flush = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")

    def ptrs(self, shape: dict):
        Z, G, D, NM = shape["Z"], shape["G"], shape["D"], shape["NM"]
        if shape["dtype"] == sj.SJ_F64:
            return [self.L, self.psi64, self.phi64]
        return [self.L, self.psi32, self.phi32]

    @staticmethod
    def working_set(shape: dict) -> int:
        esz = 8 if shape["dtype"] == sj.SJ_F64 else 4
        return (shape["D"] + shape["NM"]) * shape["G"] * shape["Z"] * esz


def spec_of(shape: dict, cand: dict) -> dict:
    spec = dict(Z=shape["Z"], G=shape["G"], D=shape["D"], NM=shape["NM"], dtype=shape["dtype"])
    spec.update(cand)
    return spec


def time_items(farm, bufs: Buffers, items, log=None, reps: int = 3):
    """items: [(shape, cand)] -> [median ms or None] (None when the specializer
    rejects the candidate)."""
    t0 = time.time()
    built = farm.specialize_many([(sj.SJ_LTIMES, spec_of(s, c)) for s, c in items], log=log)
    if log:
        log(f"compiled {len(items)} specializations in {time.time() - t0:.1f}s")
    out = []
    t0 = time.time()
    for i, ((shape, cand), (h, _, err)) in enumerate(zip(items, built)):
        if h is None:
            out.append(None)
            continue
        flush = bufs.flush if Buffers.working_set(shape) < (512 << 20) else None
        t = sj.sj_time_run(h, bufs.ptrs(shape), warmup=1, reps=reps, flush=flush)
        out.append(float(np.median(t)))
        if log and (i + 1) % 500 == 0:
            log(f"timed {i + 1}/{len(items)} ({time.time() - t0:.1f}s)")
    return out


# ------------------------------------------------------------------ the model

class MLP:
    """features -> WIDTH -> WIDTH -> 1 (ReLU), FP32 parameters on the GPU.
    Every arithmetic step runs in the library's kernels; torch only holds
    device memory."""

    def __init__(self, nfeat: int = NFEAT, width: int = WIDTH, seed: int = 0):
        import torch
        self.F, self.H = nfeat, width
        self.P = width * nfeat + width * width + 3 * width + 1
        rng = np.random.default_rng(seed)
        theta = np.zeros(self.P, dtype=np.float32)
        o = 0
        for fan_in, n_w, n_b in ((nfeat, width * nfeat, width), (width, width * width, width), (width, width, 1)):
            lim = math.sqrt(6.0 / fan_in)
            theta[o:o + n_w] = rng.uniform(-lim, lim, n_w)
            o += n_w + n_b
        self.theta = torch.from_numpy(theta).cuda()
        self.m = torch.zeros(self.P, dtype=torch.float32, device="cuda")
        self.v = torch.zeros(self.P, dtype=torch.float32, device="cuda")
        self.step = 0
        self._adam = sj.sj_specialize(sj.SJ_ADAM, dtype=sj.SJ_F32, rows=self.P)
        self._fwd = {}
        self._bwd = {}

    def _h_fwd(self, rows):
        if rows not in self._fwd:
            self._fwd[rows] = sj.sj_specialize(sj.SJ_MLP_FWD, dtype=sj.SJ_F32, rows=rows, inputs=self.F,
                                               width=self.H)
        return self._fwd[rows]

    def _h_bwd(self, rows):
        if rows not in self._bwd:
            self._bwd[rows] = sj.sj_specialize(sj.SJ_MLP_BWD, dtype=sj.SJ_F32, rows=rows, inputs=self.F,
                                               width=self.H)
        return self._bwd[rows]

    def predict(self, X: np.ndarray) -> np.ndarray:
        import torch
        X = np.ascontiguousarray(X, dtype=np.float32)
        x_d = torch.from_numpy(X).cuda()
        y_d = torch.empty(X.shape[0], dtype=torch.float32, device="cuda")
        sj.sj_run(self._h_fwd(X.shape[0]), [self.theta, x_d, y_d])
        return y_d.cpu().numpy()

    def fit(self, X: np.ndarray, y: np.ndarray, epochs: int = 300, batch: int = 128, lr: float = 2e-3,
            seed: int = 0, log=None):
        import torch
        X = np.ascontiguousarray(X, dtype=np.float32)
        y = np.ascontiguousarray(y, dtype=np.float32)
        n = X.shape[0]
        nb = n // batch
        rng = np.random.default_rng(seed)
        grad = torch.empty(self.P, dtype=torch.float32, device="cuda")
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        ws = torch.empty(batch * (4 * self.H + 2), dtype=torch.float32, device="cuda")
        hb = self._h_bwd(batch)
        losses = []
        for ep in range(epochs):
            perm = rng.permutation(n)[:nb * batch]
            xb = torch.from_numpy(X[perm]).cuda()
            yb = torch.from_numpy(y[perm]).cuda()
            for b in range(nb):
                sj.sj_run(hb, [self.theta, xb[b * batch:(b + 1) * batch], yb[b * batch:(b + 1) * batch], grad,
                               loss, ws])
                self.step += 1
                sj.sj_run_adam(self._adam, [self.theta, grad, self.m, self.v], self.step, lr=lr)
            losses.append(float(loss.item()))     # loss of the epoch's last minibatch (before its update)
            if log and (ep % 50 == 0 or ep == epochs - 1):
                log(f"epoch {ep}: train mse {losses[-1]:.4f}")
        return losses


class Picker:
    """Standardized features and log-time targets around an MLP."""

    def __init__(self, seed: int = 0):
        self.mlp = MLP(seed=seed)
        self.mu = np.zeros(NFEAT)
        self.sd = np.ones(NFEAT)
        self.tmu = 0.0
        self.tsd = 1.0

    def _norm(self, F):
        return (F - self.mu) / self.sd

    def fit(self, shapes_cands, times_ms, epochs=300, log=None):
        F = np.stack([features(s, c) for s, c in shapes_cands])
        self.mu = F.mean(axis=0)
        self.sd = F.std(axis=0)
        self.sd[self.sd < 1e-9] = 1.0
        self.mu[NFEAT - 1] = 0.0     # keep the constant feature
        t = np.log(np.asarray(times_ms, dtype=np.float64))
        self.tmu, self.tsd = float(t.mean()), float(t.std() or 1.0)
        return self.mlp.fit(self._norm(F), (t - self.tmu) / self.tsd, epochs=epochs, log=log)

    def predict_ms(self, shape, cands) -> np.ndarray:
        F = np.stack([features(shape, c) for c in cands])
        return np.exp(self.mlp.predict(self._norm(F)) * self.tsd + self.tmu)

    def pick(self, shape, cands=None):
        cands = candidates(shape) if cands is None else cands
        pred = self.predict_ms(shape, cands)
        i = int(np.argmin(pred))          # ties: lowest candidate index
        return cands[i], pred

    def save(self, path):
        with open(path, "w") as f:
            json.dump(dict(theta=self.mlp.theta.cpu().numpy().tolist(), mu=self.mu.tolist(), sd=self.sd.tolist(),
                           tmu=self.tmu, tsd=self.tsd, nfeat=NFEAT, width=WIDTH), f)

    def load(self, path):
        import torch
        with open(path) as f:
            d = json.load(f)
        self.mlp.theta = torch.tensor(d["theta"], dtype=torch.float32, device="cuda")
        self.mu, self.sd = np.array(d["mu"]), np.array(d["sd"])
        self.tmu, self.tsd = d["tmu"], d["tsd"]


def run_experiment(n_train_shapes=500, per_shape=4, n_eval=200, seed=0, workers=8, epochs=300, log=print,
                   max_k=64):
    """Collect training timings, train the picker, evaluate regret on held-out
    shapes against the exhaustive tuner's best, and the gain over the
    untuned default.  Returns a result dict."""
    from .farm import CompileFarm
    rng = np.random.default_rng(seed)

    def draw(n):
        out = []
        while len(out) < n:
            s = sample_shape(rng)
            k = round(s["Z"] ** (1 / 3))
            if k <= max_k:
                out.append(s)
        return out
    train_shapes = draw(n_train_shapes)
    eval_shapes = draw(n_eval)
    allshapes = train_shapes + eval_shapes
    max_psi = max((s["D"]) * s["G"] * s["Z"] for s in allshapes)
    max_phi = max(s["NM"] * s["G"] * s["Z"] for s in allshapes)
    bufs = Buffers(max_psi, max_phi, 256 * 64)
    res = {}
    with CompileFarm(workers) as farm:
        items = []
        for s in train_shapes:
            cs = candidates(s)
            for j in rng.choice(len(cs), size=min(per_shape, len(cs)), replace=False):
                items.append((s, cs[int(j)]))
        t0 = time.time()
        times = time_items(farm, bufs, items, log=log)
        res["train_collect_s"] = round(time.time() - t0, 1)
        pairs = [(it, t) for it, t in zip(items, times) if t is not None]
        log(f"training samples: {len(pairs)}")
        picker = Picker(seed=seed)
        t0 = time.time()
        losses = picker.fit([p[0] for p in pairs], [p[1] for p in pairs], epochs=epochs, log=log)
        res["train_s"] = round(time.time() - t0, 2)
        res["final_train_mse"] = round(losses[-1], 4)
        ev_items, owner = [], []
        for i, s in enumerate(eval_shapes):
            for c in candidates(s):
                ev_items.append((s, c))
                owner.append(i)
            ev_items.append((s, default_candidate(s)))
            owner.append(-1 - i)
        t0 = time.time()
        ev_times = time_items(farm, bufs, ev_items, log=log)
        res["eval_collect_s"] = round(time.time() - t0, 1)
    regrets, regrets2, gains, picks_ok = [], [], [], 0
    for i, s in enumerate(eval_shapes):
        cs = [(c, t) for (ss, c), o, t in zip(ev_items, owner, ev_times) if o == i and t is not None]
        dflt = [t for (ss, c), o, t in zip(ev_items, owner, ev_times) if o == -1 - i and t is not None]
        if not cs or not dflt:
            continue
        cands = [c for c, _ in cs]
        best = min(t for _, t in cs)
        pick, pred = picker.pick(s, cands)
        t_of = dict((json.dumps(c, sort_keys=True), t) for c, t in cs)
        t_pick = t_of[json.dumps(pick, sort_keys=True)]
        regrets.append(t_pick / best - 1.0)
        # top-2: compile and time the two best-predicted candidates, keep the faster
        two = np.argsort(pred, kind="stable")[:2]
        regrets2.append(min(t_of[json.dumps(cands[int(j)], sort_keys=True)] for j in two) / best - 1.0)
        gains.append(dflt[0] / t_pick)
        picks_ok += 1
    r = np.array(regrets)
    g = np.array(gains)
    res.update(dict(
        eval_shapes=picks_ok, candidates_mean=round(len(ev_items) / max(1, n_eval) - 1, 1),
        regret_mean=round(float(r.mean()), 4), regret_median=round(float(np.median(r)), 4),
        regret_p90=round(float(np.quantile(r, 0.9)), 4), regret_max=round(float(r.max()), 4),
        within_10pct=round(float(np.mean(r <= 0.10)), 4),
        top2_regret_mean=round(float(np.mean(regrets2)), 4),
        top2_regret_p90=round(float(np.quantile(regrets2, 0.9)), 4),
        speedup_vs_default_geomean=round(float(np.exp(np.mean(np.log(g)))), 4),
        speedup_vs_default_mean=round(float(g.mean()), 4),
        train_samples=len(pairs)))
    return res, picker
