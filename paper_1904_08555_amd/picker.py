"""Learned specialization picker (cost model) and its evaluation.

The exhaustive autotuner compiles and times every candidate specialization
C(s) of a shape s; the picker instead predicts each candidate's run time
relative to the shape's other candidates and compiles only the predicted best.
Five networks (features -> 64 -> 64 -> 1, ReLU, FP32, different seeds) are
averaged; each is trained on GPU with the library's own kernels
(SJ_MLP_BWD for the loss gradient, SJ_ADAM for the update, SJ_MLP_FWD for
prediction), on timings the library itself gathers with sj_time_run.  This is
the profile-guided, adaptive specialization named as future work in ClangJIT
section 6.

Shapes (LTimes): Z = k^3 with k ~ U{8..64}, G ~ U{8..128}, D = 8 U{2..32},
NM ~ U{4, 9, 16, 36, 64}, dtype ~ U{FP64, BF16x3}.  Candidates:
  FP64, column axis innermost (DGZ, DZG, GDZ, ZDG): DIRECT, tile_n in {1, 2},
      order in {ascending, rotated}, unroll 8, block 256; FP64-MFMA columns
      with default tiles, order in {ascending, rotated};
  FP64, D innermost (GZD, ZGD): FP64-MFMA rows, tile_n in {1, 2, 4}, block
      256, default operand path (LDS-staged runs where they fit);
  BF16x3 (column layouts only): columns per lane in {1, 4} (4 when it
      divides the contiguous extent), block 256.
The cost of a candidate is the median of 5 timed launches of one LTimes (after
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
NFEAT = 30
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


def resolved(shape: dict, cand: dict) -> dict:
    """The tile parameters the specializer resolves for a candidate (its
    defaults restated for LTimes), so that features see what will run."""
    Z, G, NM = shape["Z"], shape["G"], shape["NM"]
    lay = cand.get("layout", "DGZ")
    I = contiguous_extent(lay, Z, G)
    B = G * Z // I
    f64 = shape["dtype"] == sj.SJ_F64
    var = cand.get("variant", 0) or (sj.SJ_VAR_MFMA if (not f64 or I == 1) else sj.SJ_VAR_DIRECT)
    ob = (NM + 15) // 16
    r = dict(I=I, B=B, variant=var, block=cand.get("block", 0) or 256, order=cand.get("order", 0))
    far = I * 8 >= (1 << 20)
    if var == sj.SJ_VAR_DIRECT:
        r["tile"] = cand.get("tile_n", 0) or (2 if I % 2 == 0 and NM <= 16 else 1)
        r["unroll"] = cand.get("unroll", 0) or 8
        r["order"] = r["order"] or (2 if far else 1)
        r["width"], r["acc"] = 1, NM * r["tile"]
    elif not f64:
        r["tile"] = cand.get("tile_n", 0) or (4 if I % 4 == 0 else 1)
        r["unroll"] = 1
        r["order"] = 1
        r["width"], r["acc"] = 32 * r["tile"], ((NM + 31) // 32) * 16 * r["tile"]
    elif I > 1:
        t = cand.get("tile_n", 0)
        if not t:
            t = 1
            for c in (4, 2):
                if I % c == 0 and ob * 4 * c <= 32:
                    t = c
                    break
        r["tile"] = t
        r["unroll"] = cand.get("unroll", 0) or max(1, min(16 // t, 32 // (ob * t)))
        r["order"] = r["order"] or (2 if far else 1)
        r["width"], r["acc"] = 16 * t, ob * 4 * t
    else:
        # row kernel: the LDS-staged form (order 2) when the rows are even and its
        # registers and LDS allow, else lanes read their operands directly (order 1)
        D = shape["D"]
        kb = (D + 15) // 16
        wreg = kb * 4 * ob <= 32
        rt = cand.get("tile_n", 0)
        block = r["block"]

        def run_ok(t):
            lds = (block // 64) * 16 * t * (max(16 * kb, NM) + 2) * 8 + (0 if wreg else kb * 4 * ob * 512)
            return D % 2 == 0 and NM % 2 == 0 and t * ob * 4 <= 96 and (8 * t * D + 63) // 64 <= 32 and lds <= 160 * 1024
        order = cand.get("order", 0)
        if order != 1 and run_ok(rt or (2 if cand.get("block", 0) in (0, 256) else 1)):
            rt, order = rt or (2 if cand.get("block", 0) in (0, 256) else 1), 2
        else:
            rt, order = rt or (2 if 8 * ob <= 96 else 1), 1
        r["tile"], r["unroll"], r["order"] = rt, 1, order
        r["width"], r["acc"] = 1, rt * ob * 4
    return r


def features(shape: dict, cand: dict) -> np.ndarray:
    """Raw (unnormalized) feature vector of NFEAT floats."""
    f = np.zeros(NFEAT, dtype=np.float64)
    Z, G, D, NM = shape["Z"], shape["G"], shape["D"], shape["NM"]
    lay = cand.get("layout", "DGZ")
    esz = 8 if shape["dtype"] == sj.SJ_F64 else 4
    r = resolved(shape, cand)
    I, B, var = r["I"], r["B"], r["variant"]
    f[0:4] = [math.log2(Z), math.log2(G), math.log2(D), math.log2(NM)]
    f[4] = 1.0 if shape["dtype"] == sj.SJ_F64 else 0.0
    f[5] = 1.0 - f[4]
    f[6 + LAYOUTS.index(lay)] = 1.0
    f[12 + (var - 1)] = 1.0
    f[15] = math.log2(r["tile"])
    f[16] = r["unroll"] / 16.0
    f[17] = r["block"] / 512.0
    f[18] = 1.0 if r["order"] == 2 else 0.0
    f[19] = math.log2(I * esz)                             # contiguous run in bytes
    f[20] = math.log2((D + NM) * G * Z * esz)             # algorithmic bytes
    f[21] = math.log2(2.0 * D * NM * G * Z)               # flops
    f[22] = math.log2(I * esz) if lay in ("DGZ", "DZG") else math.log2(Z * esz)  # row stride proxy
    f[23] = 1.0
    w = r["width"]
    f[24] = I / (((I + w - 1) // w) * w)                  # share of lanes with a real column
    f[25] = math.log2(B)
    f[26] = math.log2(r["acc"])                            # accumulators per lane
    f[27] = 1.0 if (var == sj.SJ_VAR_MFMA and shape["dtype"] == sj.SJ_F64 and I > 1) else 0.0
    f[28] = 1.0 if I == 1 else 0.0
    f[29] = math.log2(I)
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


def time_items(farm, bufs: Buffers, items, log=None, reps: int = 5):
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

    def _check_rows(self, X):
        # the kernels read rows of exactly self.F floats: a wider or narrower
        # array would be read past its end or misaligned
        if X.ndim != 2 or X.shape[1] != self.F:
            raise ValueError(f"feature rows must have {self.F} columns, got shape {X.shape}")

    def predict(self, X: np.ndarray) -> np.ndarray:
        import torch
        X = np.ascontiguousarray(X, dtype=np.float32)
        self._check_rows(X)
        x_d = torch.from_numpy(X).cuda()
        y_d = torch.empty(X.shape[0], dtype=torch.float32, device="cuda")
        sj.sj_run(self._h_fwd(X.shape[0]), [self.theta, x_d, y_d])
        return y_d.cpu().numpy()

    def fit(self, X: np.ndarray, y: np.ndarray, epochs: int = 300, batch: int = 128, lr: float = 2e-3,
            seed: int = 0, log=None):
        import torch
        X = np.ascontiguousarray(X, dtype=np.float32)
        y = np.ascontiguousarray(y, dtype=np.float32)
        self._check_rows(X)
        n = X.shape[0]
        if y.shape != (n,) or n < batch:
            raise ValueError(f"need one target per row and at least {batch} rows, got X {X.shape}, y {y.shape}")
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
    """An ensemble of MLPs over standardized features.  The target of a training
    timing is its log-time relative to the mean log-time of the candidates
    timed for the same shape: the pick only compares candidates of one shape,
    so the network is not asked to learn the (much larger) differences between
    shapes.  Predictions are relative log-times; the pick is their argmin."""

    def __init__(self, seed: int = 0, members: int = 5):
        self.mlps = [MLP(seed=seed + 101 * k) for k in range(members)]
        self.mu = np.zeros(NFEAT)
        self.sd = np.ones(NFEAT)
        self.tsd = 1.0

    def _norm(self, F):
        return (F - self.mu) / self.sd

    @staticmethod
    def relative_targets(shapes_cands, times_ms):
        """log t minus the mean log t of the same shape's timed candidates; None
        for shapes with fewer than two timed candidates."""
        groups = {}
        for i, (s, _) in enumerate(shapes_cands):
            groups.setdefault(json.dumps(s, sort_keys=True), []).append(i)
        out = [None] * len(times_ms)
        for idx in groups.values():
            if len(idx) < 2:
                continue
            lt = np.log(np.array([times_ms[i] for i in idx], dtype=np.float64))
            for i, v in zip(idx, lt - lt.mean()):
                out[i] = float(v)
        return out

    def fit(self, shapes_cands, times_ms, epochs=200, batch=64, log=None):
        rel = self.relative_targets(shapes_cands, times_ms)
        keep = [i for i, r in enumerate(rel) if r is not None]
        F = np.stack([features(*shapes_cands[i]) for i in keep])
        t = np.array([rel[i] for i in keep])
        self.mu = F.mean(axis=0)
        self.sd = F.std(axis=0)
        self.sd[self.sd < 1e-9] = 1.0
        self.mu[NFEAT - 1] = 0.0     # keep the constant feature
        self.tsd = float(t.std() or 1.0)
        losses = []
        for k, m in enumerate(self.mlps):
            losses = m.fit(self._norm(F), t / self.tsd, epochs=epochs, batch=batch, seed=k, log=log if k == 0 else None)
        return losses

    def predict_rel(self, shape, cands) -> np.ndarray:
        F = self._norm(np.stack([features(shape, c) for c in cands]))
        return np.mean([m.predict(F) for m in self.mlps], axis=0) * self.tsd

    def pick(self, shape, cands=None):
        cands = candidates(shape) if cands is None else cands
        pred = self.predict_rel(shape, cands)
        i = int(np.argmin(pred))          # ties: lowest candidate index
        return cands[i], pred

    def save(self, path):
        with open(path, "w") as f:
            json.dump(dict(thetas=[m.theta.cpu().numpy().tolist() for m in self.mlps], mu=self.mu.tolist(),
                           sd=self.sd.tolist(), tsd=self.tsd, nfeat=NFEAT, width=WIDTH), f)

    def load(self, path):
        import torch
        with open(path) as f:
            d = json.load(f)
        self.mlps = [MLP() for _ in d["thetas"]]
        for m, th in zip(self.mlps, d["thetas"]):
            m.theta = torch.tensor(th, dtype=torch.float32, device="cuda")
        self.mu, self.sd = np.array(d["mu"]), np.array(d["sd"])
        self.tsd = d["tsd"]


def run_experiment(n_train_shapes=500, per_shape=4, n_eval=200, seed=0, workers=8, epochs=300, log=print,
                   max_k=64, dump=None):
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
    per_shape_rows = []
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
        per_shape_rows.append(dict(shape=s, times=[(c, t) for c, t in cs], pred=[float(x) for x in pred],
                                   pick=pick, default_ms=dflt[0]))
        gains.append(dflt[0] / t_pick)
        picks_ok += 1
    if dump:
        with open(dump, "w") as f:
            json.dump(dict(train=[(sc[0], sc[1], t) for sc, t in pairs], eval=per_shape_rows), f)
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
