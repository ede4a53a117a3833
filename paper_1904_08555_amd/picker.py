"""Learned specialization picker (cost model) and its evaluation.

The exhaustive autotuner (tune.py) compiles and times every candidate
specialization of a shape; the picker predicts each candidate's run time
relative to the shape's other candidates and compiles only what it cannot rule
out.  The candidate set of a shape s is exactly the tuner's: C(s) = the union
over nestings of tune.candidates(LTimes, nesting, s), so the tuner's best over C(s) is both
the measure of the picker's regret and its fallback.

Model: five networks (features -> 64 -> 64 -> 1, ReLU, FP32, different seeds);
each is trained on the GPU with the library's own kernels (SJ_MLP_BWD for the
loss gradient, SJ_ADAM for the update, SJ_MLP_FWD for prediction), on timings
the library gathers with sj_time_run.  The features describe the
specialization the request resolves to (sj_resolve: the tiles, structure and
load/store forms that will run), so the network sees what the compiler gets.

Decision with fallback: rank C(s) by the ensemble mean; the candidates whose
predicted advantage over the first is within the ensemble's spread
(mean_c - mean_best < TAU * (sd_c + sd_best)) cannot be told apart by the
model, so the first K of them (K <= KMAX) are compiled and timed, exactly as
the tuner would time them, and the fastest is kept.  With a confident model
that is one compile; at worst KMAX instead of |C(s)|.  This is the
profile-guided, adaptive specialization named as future work in ClangJIT
section 6.

Shapes (LTimes): Z = k^3 with k ~ U{8..64}, G ~ U{8..128}, D = 8 U{2..32},
NM ~ U{4, 9, 16, 36, 64}, dtype ~ U{FP64, BF16x3}.  The cost of a candidate
is the median of 5 timed launches of one LTimes (after one warm-up), with L2
and the last-level cache flushed first when the working set is under 512 MB.
Regret of a choice: t(choice) / min_{c in C(s)} t(c) - 1.
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np

from . import sj, tune

LAYOUTS = sj.LAYOUTS
COLUMN_LAYOUTS = ("DGZ", "DZG", "GDZ", "ZDG")
NFEAT = 37
WIDTH = 64
TAU = 1.0      # spread multiple within which two predictions are not told apart
KMAX = 4       # at most this many candidates compiled and timed per shape


def sample_shape(rng: np.random.Generator) -> dict:
    k = int(rng.integers(8, 65))
    return dict(Z=k ** 3, G=int(rng.integers(8, 129)), D=8 * int(rng.integers(2, 33)),
                NM=int(rng.choice([4, 9, 16, 36, 64])),
                dtype=int(rng.choice([sj.SJ_F64, sj.SJ_BF16X3])))


def contiguous_extent(layout: str, Z: int, G: int) -> int:
    return tune.contiguous_extent(layout, Z, G)


def candidates(shape: dict, layouts=None) -> list:
    """C(s): the exhaustive tuner's candidates over every nesting (restricted
    to ``layouts`` when given), each tagged with its nesting; candidates the
    specializer refuses for the shape are left out."""
    lays = list(layouts or LAYOUTS)
    out = []
    for lay in lays:
        for c in tune.candidates(sj.SJ_LTIMES, lay, shape["Z"], shape["G"], shape["D"], shape["NM"],
                                 shape["dtype"]):
            cand = dict(layout=lay, **c)
            try:
                sj.sj_resolve(sj.SJ_LTIMES, **spec_of(shape, cand))
            except sj.SJError:
                continue
            out.append(cand)
    return out


def default_candidate(shape: dict) -> dict:
    """What a caller gets without tuning: Kripke's default nesting DGZ with the
    library's default tile parameters."""
    return dict(layout="DGZ")


def spec_of(shape: dict, cand: dict) -> dict:
    spec = dict(Z=shape["Z"], G=shape["G"], D=shape["D"], NM=shape["NM"], dtype=shape["dtype"])
    spec.update(cand)
    return spec


def features(shape: dict, cand: dict) -> np.ndarray:
    """Raw (unnormalized) feature vector of NFEAT floats, computed from the
    specialization the request resolves to."""
    r = sj.sj_resolve(sj.SJ_LTIMES, **spec_of(shape, cand))
    f = np.zeros(NFEAT, dtype=np.float64)
    Z, G, D, NM = shape["Z"], shape["G"], shape["D"], shape["NM"]
    lay = LAYOUTS[r["layout"]]
    f64 = shape["dtype"] == sj.SJ_F64
    esz = 8 if f64 else 4
    I = contiguous_extent(lay, Z, G)
    B = G * Z // I
    var, tn, blk = r["variant"], max(1, r["tile_n"]), r["block"]
    col_mfma = var == sj.SJ_VAR_MFMA and f64 and I > 1
    row_mfma = var == sj.SJ_VAR_MFMA and f64 and I == 1
    f[0:4] = [math.log2(Z), math.log2(G), math.log2(D), math.log2(NM)]
    f[4] = 1.0 if f64 else 0.0
    f[5] = 1.0 - f[4]
    f[6 + LAYOUTS.index(lay)] = 1.0
    f[12 + (var - 1)] = 1.0                               # DIRECT, STAGED, MFMA
    f[15] = 1.0 if col_mfma else 0.0
    f[16] = 1.0 if row_mfma else 0.0
    if var == sj.SJ_VAR_STAGED:
        tile, width, acc = tn // blk, 1, NM * (tn // blk)
    elif var == sj.SJ_VAR_DIRECT:
        tile, width, acc = tn, tn, NM * tn
    elif not f64:
        tile, width, acc = tn, 32 * tn, ((NM + 31) // 32) * 16 * tn
    elif col_mfma:
        tile, width, acc = tn, 16 * tn, ((NM + 15) // 16) * 4 * tn
    else:
        tile, width, acc = tn, 1, tn * ((NM + 15) // 16) * 4
    f[17] = math.log2(tile)
    f[18] = r["unroll"] / 16.0
    f[19] = blk / 512.0
    f[20] = 1.0 if r["order"] == 2 else 0.0
    f[21] = 1.0 if r["flags"] & sj.SJ_FLAG_LOADS_NONTEMPORAL else 0.0
    f[22] = 1.0 if r["flags"] & sj.SJ_FLAG_STORES_NONTEMPORAL else 0.0
    f[23] = math.log2(I * esz)                            # contiguous run in bytes
    f[24] = math.log2((D + NM) * G * Z * esz)             # algorithmic bytes
    f[25] = math.log2(2.0 * D * NM * G * Z)               # flops
    f[26] = math.log2(I * esz) if lay in ("DGZ", "DZG") else math.log2(Z * esz)  # row stride proxy
    f[27] = I / (((I + width - 1) // width) * width) if width > 1 else 1.0       # lanes holding a real column
    f[28] = math.log2(B)
    f[29] = math.log2(max(1, acc))                        # accumulators per lane
    f[30] = r["tile_k"] / 32.0 if var == sj.SJ_VAR_STAGED else 0.0
    f[31] = math.log2(I)
    f[32] = math.log2(max(1.0, G * Z / max(1, width)))    # lanes of work
    f[33] = 1.0 if r["flags"] & sj.SJ_FLAG_INDEX64 else 0.0
    f[34] = math.log2(2.0 * D * NM * G * Z) - math.log2((D + NM) * G * Z * esz)  # arithmetic intensity
    f[35] = 1.0 if r["flags"] & sj.SJ_FLAG_XCD_CONTIGUOUS else 0.0
    f[36] = 1.0
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
        if shape["dtype"] == sj.SJ_F64:
            return [self.L, self.psi64, self.phi64]
        return [self.L, self.psi32, self.phi32]

    @staticmethod
    def working_set(shape: dict) -> int:
        esz = 8 if shape["dtype"] == sj.SJ_F64 else 4
        return (shape["D"] + shape["NM"]) * shape["G"] * shape["Z"] * esz

    @staticmethod
    def for_shapes(shapes):
        return Buffers(max(s["D"] * s["G"] * s["Z"] for s in shapes),
                       max(s["NM"] * s["G"] * s["Z"] for s in shapes), 256 * 64)


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
    timed for the same shape: a decision only compares candidates of one
    shape, so the network is not asked to learn the (much larger) differences
    between shapes.  Predictions are relative log-times."""

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

    def predict_members(self, shape, cands) -> np.ndarray:
        """(members, len(cands)) relative log-time predictions."""
        F = self._norm(np.stack([features(shape, c) for c in cands]))
        return np.stack([m.predict(F) for m in self.mlps]).astype(np.float64) * self.tsd

    def predict_rel(self, shape, cands) -> np.ndarray:
        return self.predict_members(shape, cands).mean(axis=0)

    def shortlist(self, shape, cands, tau: float = TAU, kmax: int = KMAX):
        """Indices of the candidates to compile and time: the predicted best,
        then (in predicted order) those the ensemble's spread cannot separate
        from it, at most kmax in all.  Returns (indices, mean predictions)."""
        pm = self.predict_members(shape, cands)
        mu, sd = pm.mean(axis=0), pm.std(axis=0)
        order = np.argsort(mu, kind="stable")          # ties: lowest candidate index
        b = order[0]
        close = [int(j) for j in order[1:] if mu[j] - mu[b] < tau * (sd[j] + sd[b])]
        return [int(b)] + close[:kmax - 1], mu

    def pick(self, shape, cands=None):
        cands = candidates(shape) if cands is None else cands
        pred = self.predict_rel(shape, cands)
        i = int(np.argmin(pred))          # ties: lowest candidate index
        return cands[i], pred

    def save(self, path):
        """The ensemble's parameters and feature scaling, as JSON or (path ending
        in .npz) a numpy archive that loads without unpickling."""
        d = dict(thetas=[m.theta.cpu().numpy().tolist() for m in self.mlps], mu=self.mu.tolist(),
                 sd=self.sd.tolist(), tsd=self.tsd, nfeat=NFEAT, width=WIDTH)
        if str(path).endswith(".npz"):
            _save_npz(d, path)
        else:
            with open(path, "w") as f:
                json.dump(d, f)

    def load(self, path):
        import torch
        d = _load_weights(path)
        self.mlps = [MLP() for _ in d["thetas"]]
        for m, th in zip(self.mlps, d["thetas"]):
            m.theta = torch.tensor(np.asarray(th, dtype=np.float32), device="cuda")
        self.mu, self.sd = np.array(d["mu"]), np.array(d["sd"])
        self.tsd = float(d["tsd"])

    @classmethod
    def pretrained(cls, path=None):
        """The ensemble trained on MI355X timings (750 shapes x 8 candidates, the
        workload of ``collect``), shipped with the package as PRETRAINED."""
        p = cls(members=0)
        p.load(path or PRETRAINED)
        return p


PRETRAINED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "picker_mi355x.npz")


def _save_npz(d, path):
    np.savez(path, thetas=np.asarray(d["thetas"], dtype=np.float32), mu=np.asarray(d["mu"], dtype=np.float64),
             sd=np.asarray(d["sd"], dtype=np.float64), tsd=np.float64(d["tsd"]), nfeat=np.int64(d["nfeat"]),
             width=np.int64(d["width"]))


def _load_weights(path):
    """Saved weights as a dict, checked against this module's network size."""
    if str(path).endswith(".npz"):
        with np.load(path, allow_pickle=False) as z:
            d = {k: z[k] for k in ("thetas", "mu", "sd", "tsd", "nfeat", "width")}
    else:
        with open(path) as f:
            d = json.load(f)
    nparams = WIDTH * NFEAT + WIDTH * WIDTH + 3 * WIDTH + 1
    if int(d["nfeat"]) != NFEAT or int(d["width"]) != WIDTH or any(len(t) != nparams for t in d["thetas"]) \
            or len(d["mu"]) != NFEAT or len(d["sd"]) != NFEAT:
        raise ValueError(f"{path}: weights of a network with {d['nfeat']} features and width {d['width']}, "
                         f"expected {NFEAT} and {WIDTH}")
    return d


def weights_to_npz(json_path, npz_path):
    """Convert weights saved as JSON to the numpy archive form (no GPU needed)."""
    _save_npz(_load_weights(json_path), npz_path)


# ------------------------------------------------------------------ the experiment

def draw_shapes(rng, n, max_k=64):
    out = []
    while len(out) < n:
        s = sample_shape(rng)
        if round(s["Z"] ** (1 / 3)) <= max_k:
            out.append(s)
    return out


def experiment_shapes(n_train_shapes, n_eval, seed=0, max_k=64, extra_train_shapes=0):
    """(training shapes, held-out shapes): n_train_shapes, then the n_eval
    held-out shapes, then extra_train_shapes more training shapes, all from one
    generator, so the held-out shapes depend only on the seed, n_train_shapes
    and max_k."""
    rng = np.random.default_rng(seed)
    train_shapes = draw_shapes(rng, n_train_shapes, max_k)
    eval_shapes = draw_shapes(rng, n_eval, max_k)
    return train_shapes + draw_shapes(rng, extra_train_shapes, max_k), eval_shapes


def collect(n_train_shapes=250, per_shape=8, n_eval=200, seed=0, workers=12, log=print, max_k=64, layouts=None,
            eval_slice=None, train=True, extra_train_shapes=0):
    """Timings for the experiment: per_shape random candidates of each training
    shape, and every candidate (the exhaustive tuner's whole set) plus the
    default of each held-out shape.  ``eval_slice`` = (lo, hi) restricts the
    held-out shapes (to split a long collection over several runs); the shapes
    themselves depend only on the seed.  ``extra_train_shapes`` more training
    shapes are drawn after the held-out ones, so that the held-out shapes do
    not depend on it.  ``train`` = False skips the training timings; "only"
    times them and no held-out shape.  Returns a JSON-able dict."""
    from .farm import CompileFarm
    train_shapes, eval_shapes = experiment_shapes(n_train_shapes, n_eval, seed, max_k, extra_train_shapes)
    crng = np.random.default_rng(seed + 1)
    items = []
    for s in train_shapes:
        cs = candidates(s, layouts)
        for j in crng.choice(len(cs), size=min(per_shape, len(cs)), replace=False):
            items.append((s, cs[int(j)]))
    lo, hi = eval_slice or (0, n_eval)
    if train == "only":
        lo = hi = 0
    ev_items = []
    for i in range(lo, hi):
        s = eval_shapes[i]
        for c in candidates(s, layouts) + [default_candidate(s)]:
            ev_items.append((i, s, c))
    used = (train_shapes if train else []) + eval_shapes[lo:hi]
    bufs = Buffers.for_shapes(used)
    out = dict(seed=seed, layouts=layouts, max_k=max_k, eval_slice=[lo, hi])
    with CompileFarm(workers) as farm:
        if train:
            t0 = time.time()
            times = time_items(farm, bufs, items, log=log)
            out["train"] = [(s, c, t) for (s, c), t in zip(items, times) if t is not None]
            out["train_collect_s"] = round(time.time() - t0, 1)
            log(f"training timings: {len(out['train'])}")
        t0 = time.time()
        ev_times = time_items(farm, bufs, [(s, c) for _, s, c in ev_items], log=log) if ev_items else []
        out["eval_collect_s"] = round(time.time() - t0, 1)
    rows = {}
    for (i, s, c), t in zip(ev_items, ev_times):
        r = rows.setdefault(i, dict(index=i, shape=s, times=[], default_ms=None))
        if c == default_candidate(s):
            r["default_ms"] = t
        elif t is not None:
            r["times"].append((c, t))
    out["eval"] = [rows[i] for i in sorted(rows)]
    del bufs
    return out


def evaluate(data, seed=0, epochs=200, log=print, tau=TAU, kmax=KMAX, picker=None):
    """Train the ensemble on data["train"] (unless ``picker`` is given) and
    score it on data["eval"] against the exhaustive tuner's best over the same
    candidate set.  Returns (result dict, picker, per-shape rows)."""
    res = {}
    if picker is None:
        pairs = [((s, c), t) for s, c, t in data["train"]]
        picker = Picker(seed=seed)
        t0 = time.time()
        losses = picker.fit([p[0] for p in pairs], [p[1] for p in pairs], epochs=epochs, log=log)
        res["train_s"] = round(time.time() - t0, 2)
        res["final_train_mse"] = round(losses[-1], 4)
        res["train_samples"] = len(pairs)
    reg1, regk, compiles, gains, gains_k, rand, ncands, dflt_reg, rows = [], [], [], [], [], [], [], [], []
    for row in data["eval"]:
        s, ct, dflt = row["shape"], row["times"], row["default_ms"]
        if len(ct) < 2 or dflt is None:
            continue
        cands = [c for c, _ in ct]
        t = np.array([x for _, x in ct])
        best = t.min()
        short, mu = picker.shortlist(s, cands, tau=tau, kmax=kmax)
        t1 = t[short[0]]
        tk = t[short].min()
        reg1.append(t1 / best - 1.0)
        regk.append(tk / best - 1.0)
        compiles.append(len(short))
        ncands.append(len(cands))
        gains.append(dflt / t1)
        gains_k.append(dflt / tk)
        rand.append(float(np.mean(t / best - 1.0)))
        dflt_reg.append(dflt / best - 1.0)
        rows.append(dict(shape=s, n_candidates=len(cands), pick=cands[short[0]], shortlist=[cands[j] for j in short],
                         best=cands[int(np.argmin(t))], t_best=float(best), t_pick=float(t1), t_shortlist=float(tk),
                         t_default=float(dflt)))

    def stats(x, name):
        x = np.array(x)
        return {f"{name}_mean": round(float(x.mean()), 4), f"{name}_median": round(float(np.median(x)), 4),
                f"{name}_p90": round(float(np.quantile(x, 0.9)), 4), f"{name}_max": round(float(x.max()), 4)}
    res.update(eval_shapes=len(reg1), candidates_mean=round(float(np.mean(ncands)), 1),
               compiles_mean=round(float(np.mean(compiles)), 2),
               compiles_saved_frac=round(1.0 - float(np.sum(compiles)) / float(np.sum(ncands)), 4))
    res.update(stats(reg1, "regret"))
    res["within_10pct"] = round(float(np.mean(np.array(reg1) <= 0.10)), 4)
    res.update(stats(regk, "shortlist_regret"))
    res["shortlist_within_10pct"] = round(float(np.mean(np.array(regk) <= 0.10)), 4)
    res.update(stats(rand, "random_choice_regret"))
    res.update(stats(dflt_reg, "default_regret"))
    res["speedup_vs_default_geomean"] = round(float(np.exp(np.mean(np.log(gains)))), 4)
    res["shortlist_speedup_vs_default_geomean"] = round(float(np.exp(np.mean(np.log(gains_k)))), 4)
    res["tau"], res["kmax"] = tau, kmax
    return res, picker, rows


def run_experiment(n_train_shapes=250, per_shape=8, n_eval=200, seed=0, workers=12, epochs=200, log=print,
                   max_k=64, layouts=None, dump=None):
    """collect() then evaluate() in one process."""
    data = collect(n_train_shapes, per_shape, n_eval, seed, workers, log, max_k, layouts)
    if dump:
        with open(dump, "w") as f:
            json.dump(data, f)
    res, picker, _ = evaluate(data, seed=seed, epochs=epochs, log=log)
    res["train_collect_s"] = data.get("train_collect_s")
    res["eval_collect_s"] = data.get("eval_collect_s")
    return res, picker
