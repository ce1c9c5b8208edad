"""Query router: the surrogate answers, the batched MPM checks and falls back.

Each query is a contact (indenter, pose, depth). Per batch of queries:
  1. the gap field kernel builds the surrogate inputs and the surrogate
     predicts the surface displacement;
  2. the out-of-distribution score is the distance from the query's feature
     vector (4 x 4 box means of the gap field in mm, i.e. 16 x 16 values,
     and the depth in mm) to its nearest training sample; queries above the
     threshold (the 99.5th percentile of the held-out samples' scores) go to
     the MPM;
  3. a seeded 2% audit sends further queries to the MPM, where the surrogate's
     height error is measured against the MPM's answer;
  4. a guard decides which queries the surrogate may answer at all, from the
     audits (applied in stream order: when the guard closes on a query's
     indenter family, every later query of the batch that the surrogate was
     going to answer for that family is solved by the MPM as well, so no
     surrogate answer leaves after the audit that closed it):
     * "breaker": a circuit breaker (per indenter family, or one for all
       queries) routes every later query to the MPM once the RMSE of its
       most recent audits exceeds the limit (5 um by default); a breaker
       starts tripped when the held-out error of its queries is above it;
     * "budget": the limit bounds the error of all served answers together.
       Queries fall into classes: the indenter family, or (with depth
       edges) the family and the press depth's bin, both known from the
       query. Each class's mean squared height error is estimated from its
       held-out samples and its audits, as an upper confidence bound (mean
       plus z standard errors, z = 1.645: one-sided 95 %); classes are
       admitted in increasing order of that bound while the mean of the
       bounds, weighted by each class's share of the queries so far, stays
       within the limit squared. The admitted set is recomputed after every
       audit and at every batch;
  5. the MPM answers every query sent to it; the rest keep the surrogate's.
Latency of a query = its batch's start -> its answer ready (all queries are
queued at time zero and batches run back to back).
"""
from __future__ import annotations

import bisect
import math
import time

import numpy as np
import torch

from . import dataset as D
from . import native
from .surrogate import Net
from .training import per_sample_rmse
from .workloads import SplitMix64

FEAT_POOL = 4


def features(x, depth_scale=1.0) -> torch.Tensor:
    """[n][(res/4)^2 + 1] router features of surrogate inputs x [n][res][res][2]."""
    n, res = x.shape[0], x.shape[1]
    gap = x[..., 0].contiguous()
    depth = x[:, 0, 0, 1].contiguous()
    out = torch.empty(n, (res // FEAT_POOL) ** 2 + 1, dtype=torch.float32, device=x.device)
    native.tsg_call("tsg_features", gap.data_ptr(), n, res, res, FEAT_POOL, depth.data_ptr(), depth_scale,
                    out.data_ptr(), torch.cuda.current_stream().cuda_stream)
    return out


def nn_distance(q, ref):
    d2 = torch.empty(q.shape[0], dtype=torch.float32, device=q.device)
    idx = torch.empty(q.shape[0], dtype=torch.int32, device=q.device)
    native.tsg_call("tsg_nn_dist", q.data_ptr(), q.shape[0], ref.data_ptr(), ref.shape[0], q.shape[1],
                    d2.data_ptr(), idx.data_ptr(), torch.cuda.current_stream().cuda_stream)
    return d2.sqrt(), idx


def query_class(contact, depth_edges=None) -> int:
    """Router class of a query: its indenter family, or with depth_edges (m,
    ascending) family * (len(edges) + 1) + the index of its depth's bin."""
    fam = int(contact["cfg"]["shape"])
    if not depth_edges:
        return fam
    return fam * (len(depth_edges) + 1) + bisect.bisect_right(list(depth_edges), float(contact["depth"]))


def audit_draws(n, rate, seed):
    """Query k is audited when the k-th SplitMix64 output of `seed` is below rate * 2^64."""
    rng = SplitMix64(seed)
    lim = int(rate * 2.0 ** 64)
    return np.array([rng.next_u64() < lim for _ in range(n)], dtype=bool)


class FamilyError:
    """Running count, sum and sum of squares of per-sample height mean
    squared errors (um^2) of one indenter family."""

    def __init__(self, n=0, mean=0.0, sd=0.0):
        self.n = int(n)
        self.s1 = self.n * float(mean)
        self.s2 = self.n * (float(sd) ** 2 + float(mean) ** 2)

    def add(self, sq):
        self.n += 1
        self.s1 += sq
        self.s2 += sq * sq

    def mean(self):
        return self.s1 / self.n if self.n else math.inf

    def upper(self, z):
        """Mean plus z standard errors of the mean; infinite without samples."""
        if self.n == 0:
            return math.inf
        m = self.s1 / self.n
        var = max(0.0, self.s2 / self.n - m * m)
        return m + z * math.sqrt(var / self.n)


def admit(bounds, shares, limit_sq):
    """Families admitted under an error budget: in increasing order of their
    error bound, the longest run whose share-weighted mean bound is at most
    limit_sq (adding a larger bound only raises the mean, so the run is a
    prefix of that order)."""
    order = sorted(bounds, key=lambda f: (bounds[f], f))
    out, w, ws = set(), 0.0, 0.0
    for f in order:
        if not math.isfinite(bounds[f]):
            break
        w1, ws1 = w + shares.get(f, 0.0) * bounds[f], ws + shares.get(f, 0.0)
        if ws1 > 0 and w1 > limit_sq * ws1:
            break
        out.add(f)
        w, ws = w1, ws1
    return out


class Router:
    """Surrogate answers with OOD and audit fallbacks to the MPM.

    policy "breaker": the circuit breaker is kept per indenter family when
    per_class is set (the query names its indenter), else one breaker covers
    every query; prior_rmse_um maps a breaker key to the surrogate's
    held-out height RMSE for its queries, and breakers whose prior exceeds
    the limit start tripped.
    policy "budget": prior_stats maps each query class (query_class with
    depth_edges) to the count, mean and standard deviation of its held-out
    samples' height mean squared error (um^2); a class without them is never
    admitted."""

    # route codes (BREAKER: the guard was closed for the query's family when
    # its batch started; BREAKER_IN_BATCH: an audit of the same batch closed it)
    SURROGATE, OOD, AUDIT, BREAKER, BREAKER_IN_BATCH = 0, 1, 2, 3, 4

    def __init__(self, net: Net, train_features, threshold, audit_rate=0.02, audit_seed=7, rmse_limit_um=5.0,
                 window=20, per_class=True, prior_rmse_um=None, policy="breaker", prior_stats=None, z=1.645,
                 depth_edges=None):
        if policy not in ("breaker", "budget"):
            raise ValueError(f"unknown router policy {policy!r}")
        self.net = net
        self.train_features = train_features.contiguous()
        self.threshold = float(threshold)
        self.audit_rate = audit_rate
        self.audit_seed = audit_seed
        self.rmse_limit_um = rmse_limit_um
        self.window = window
        self.per_class = per_class or policy == "budget"
        self.prior_rmse_um = {int(k): float(v) for k, v in (prior_rmse_um or {}).items()}
        self.policy = policy
        self.prior_stats = {int(k): dict(v) for k, v in (prior_stats or {}).items()}
        self.z = z
        self.depth_edges = [float(e) for e in depth_edges] if depth_edges else None

    @staticmethod
    def calibrate(train_features, heldout_features, q=0.995):
        d, _ = nn_distance(heldout_features.contiguous(), train_features.contiguous())
        return float(torch.quantile(d.cpu(), q))

    def _over_limit(self, sq):
        recent = sq[-self.window:]
        return math.sqrt(sum(recent) / len(recent)) > self.rmse_limit_um

    def serve(self, contacts, batch=512, log=None):
        """Answer every contact; returns (answers [n][res][res][3] in Y_UNIT,
        report dict, route code per query)."""
        n = len(contacts)
        audit = audit_draws(n, self.audit_rate, self.audit_seed)
        key = np.array([query_class(c, self.depth_edges) if self.per_class else 0 for c in contacts])
        answers = torch.empty(n, D.RES, D.RES, 3, dtype=torch.float32, device="cuda")
        lat = np.zeros(n)
        route = np.zeros(n, dtype=np.int8)
        audits_sq = {}
        budget = self.policy == "budget"
        fams = sorted(set(int(k) for k in np.unique(key)) | set(self.prior_stats))
        err = {f: FamilyError(**{k: self.prior_stats[f][k] for k in ("n", "mean", "sd")})
               if f in self.prior_stats else FamilyError() for f in fams}
        seen = {f: 0 for f in fams}

        def admitted_now():
            tot = sum(seen.values())
            shares = {f: seen[f] / tot if tot else 1.0 / len(fams) for f in fams}
            return admit({f: err[f].upper(self.z) for f in fams}, shares, self.rmse_limit_um ** 2)

        if budget:
            closed = set()
        else:
            closed = {k for k, e in self.prior_rmse_um.items() if e > self.rmse_limit_um} if self.per_class else set()
        closed_at_start = None
        admitted_log = []
        n_mpm = 0
        torch.cuda.synchronize()
        t_all = time.perf_counter()
        for k0 in range(0, n, batch):
            cs = contacts[k0:k0 + batch]
            m = len(cs)
            kb = key[k0:k0 + m]
            rb = route[k0:k0 + m]  # view
            t0 = time.perf_counter()
            if budget:
                for f in kb:
                    seen[int(f)] += 1
                closed = set(fams) - admitted_now()
                admitted_log.append((k0, sorted(set(fams) - closed)))
            if closed_at_start is None:
                closed_at_start = sorted(closed)
            brk = np.array([k in closed for k in kb], dtype=bool)
            x = D.inputs(cs)
            pred = None
            send = brk.copy()
            if not brk.all():
                pred = self.net.forward(x).clone()
                d, _ = nn_distance(features(x), self.train_features)
                ood = (d > self.threshold).cpu().numpy() & ~brk
                aud = audit[k0:k0 + m] & ~brk & ~ood
                send |= ood | aud
                rb[ood] = self.OOD
                rb[aud] = self.AUDIT
                answers[k0:k0 + m] = pred
            rb[brk] = self.BREAKER
            torch.cuda.synchronize()
            lat[k0:k0 + m] = time.perf_counter() - t0
            idx = np.nonzero(send)[0]
            late = []
            if len(idx):
                ym = D.solve([cs[i] for i in idx])
                n_mpm += len(idx)
                it = torch.tensor(idx, device="cuda")
                aud_idx = [j for j, i in enumerate(idx) if rb[i] == self.AUDIT]
                if aud_idx:
                    ai = torch.tensor(aud_idx, device="cuda")
                    e = per_sample_rmse(pred.index_select(0, it.index_select(0, ai)), ym.index_select(0, ai), 2)
                    # audits in stream order: a guard that closes re-routes the
                    # later surrogate answers of its family in this batch
                    for j, v in zip(aud_idx, (e * D.Y_UNIT * 1e6).cpu().tolist()):
                        kk = int(kb[idx[j]])
                        sq = audits_sq.setdefault(kk, [])
                        sq.append(v * v)
                        if budget:
                            err[kk].add(v * v)
                            newly = (set(fams) - admitted_now()) - closed
                            admitted_log.append((k0 + int(idx[j]), sorted(set(fams) - closed - newly)))
                        else:
                            newly = {kk} if kk not in closed and self._over_limit(sq) else set()
                        closed |= newly
                        if newly:
                            late += [i for i in range(idx[j] + 1, m) if kb[i] in newly and rb[i] == self.SURROGATE]
                answers.index_copy_(0, it + k0, ym)
                torch.cuda.synchronize()
                lat[k0 + idx] = time.perf_counter() - t0
            if late:
                late = np.array(sorted(set(late)))
                yl = D.solve([cs[i] for i in late])
                n_mpm += len(late)
                answers.index_copy_(0, torch.tensor(late, device="cuda") + k0, yl)
                rb[late] = self.BREAKER_IN_BATCH
                torch.cuda.synchronize()
                lat[k0 + late] = time.perf_counter() - t0
            if log:
                log(f"router: {k0 + m}/{n} answered, {n_mpm} by MPM, closed={sorted(closed)}")
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_all
        all_sq = [v for sq in audits_sq.values() for v in sq]
        audited = math.sqrt(sum(all_sq) / len(all_sq)) if all_sq else float("nan")
        rep = {
            "policy": self.policy, "depth_edges_m": self.depth_edges, "queries": n, "wall_s": wall, "frames_per_s": n / wall,
            "latency_p50_ms": float(np.percentile(lat, 50) * 1e3),
            "latency_p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mpm_fallbacks": int(n_mpm), "ood": int((route == self.OOD).sum()),
            "audited": int((route == self.AUDIT).sum()),
            "breaker_routed": int((route == self.BREAKER).sum()),
            "breaker_rerouted_in_batch": int((route == self.BREAKER_IN_BATCH).sum()),
            "breaker_tripped_at_start": [int(k) for k in (closed_at_start or [])],
            "breaker_tripped": sorted(int(k) for k in closed),
            "served_by_surrogate": int((route == self.SURROGATE).sum()),
            "audited_height_rmse_um": audited,
            "prior_rmse_um": {str(k): v for k, v in sorted(self.prior_rmse_um.items())},
            "per_class": {str(int(k)): {"queries": int((key == k).sum()),
                                        "surrogate": int(((key == k) & (route == self.SURROGATE)).sum()),
                                        "audits": len(audits_sq.get(int(k), [])),
                                        "audited_rmse_um": (math.sqrt(sum(audits_sq[int(k)]) / len(audits_sq[int(k)]))
                                                            if audits_sq.get(int(k)) else None),
                                        "tripped": int(k) in closed,
                                        "tripped_at_start": int(k) in (closed_at_start or [])}
                          for k in np.unique(key)},
        }
        if budget:
            served = [f for f in fams if f not in closed]
            tot = sum(seen.values())
            for f in fams:
                pc = rep["per_class"].setdefault(str(f), {})
                pc["error_bound_um2"] = err[f].upper(self.z)
                pc["error_mean_um2"] = err[f].mean()
                pc["error_samples"] = err[f].n
            ws = sum(seen[f] for f in served)
            rep["budget"] = {
                "limit_um": self.rmse_limit_um, "z": self.z,
                "admitted_at_end": served,
                "bound_rmse_um_of_admitted": (math.sqrt(sum(seen[f] * err[f].upper(self.z) for f in served) / ws)
                                              if ws else None),
                "expected_rmse_um_of_admitted": (math.sqrt(sum(seen[f] * err[f].mean() for f in served) / ws)
                                                 if ws else None),
                "changes": [(int(i), a) for (i, a), prev in zip(admitted_log, [None] + admitted_log[:-1])
                            if prev is None or prev[1] != a],
                "shares": {str(f): seen[f] / tot for f in fams} if tot else {}}
        return answers, rep, route


def plain_mpm(contacts, batch=512, log=None):
    """Answer every contact with the batched MPM alone; (answers, report)."""
    n = len(contacts)
    lat = np.zeros(n)
    outs = []
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for k0 in range(0, n, batch):
        cs = contacts[k0:k0 + batch]
        t0 = time.perf_counter()
        outs.append(D.solve(cs))
        torch.cuda.synchronize()
        lat[k0:k0 + len(cs)] = time.perf_counter() - t0
        if log:
            log(f"plain MPM: {k0 + len(cs)}/{n} answered")
    wall = time.perf_counter() - t_all
    return torch.cat(outs), {"queries": n, "wall_s": wall, "frames_per_s": n / wall,
                             "latency_p50_ms": float(np.percentile(lat, 50) * 1e3),
                             "latency_p99_ms": float(np.percentile(lat, 99) * 1e3)}
