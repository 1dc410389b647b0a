"""Serving loop: requests of mixed d, N, T and tolerance, admitted by an HBM
budget and solved with continuous batching over the library's batch entry
points (lgp_batch_*).

Every request is built on arrival (operator, ILU(0) factor in FP64, load
vector) once its device bytes (from the library's size queries) fit in the
budget next to those of the requests in flight; it then takes a slot in the
batch of its grid shape and pattern (a new batch when none has a free
slot). The scheduler advances every batch with running requests by a few
PCG iterations per round, on one stream, so requests that arrive while
others run join their batch at the next round and leave it when they
converge; their buffers are released at once. Each request's result is the
one lgp_pcg_solve gives it alone, bit for bit (the batch computes exactly
that per request).

A request is a dict with d, N, T, J, seed, tol (synth.serving_requests);
coefficients a = 2 + sum c_j L_j..., b = 1 + |x|^2, f from the manufactured
solution (the synthetic family), evaluated by paper_2004_13961_amd.workload.
"""
from __future__ import annotations

import collections
import time

import numpy as np
import torch

from . import lgpcg
from .lgpcg import lib
from .solver import Batch, Factor, Problem
from .workload import family_nodal


def _vector_bytes(n: int) -> int:
    # load vector and solution, and the request's slot of a batch workspace
    return 2 * n * 8 + 6 * n * 8


class Server:
    def __init__(self, budget_bytes: int, slots_per_batch: int = 8, step_iters: int = 2,
                 stream: torch.cuda.Stream = None):
        self.budget = int(budget_bytes)
        self.slots = slots_per_batch
        self.step_iters = step_iters
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.batches = collections.defaultdict(list)   # key -> [Batch]
        self.used = 0

    def _key(self, P: Problem, M: Factor):
        desc = M.describe()
        return (P.d, P.N, tuple(desc["offsets"]))

    def _prepare(self, rec):
        """Operator of an arrived request (small) and the exact device bytes
        its factor will take (size query on that operator)."""
        r = rec["req"]
        d, N = r["d"], r["N"]
        with torch.cuda.stream(self.stream):
            a, b, f, _ = family_nodal(d, N, r["J"], r["seed"])
            dev = lambda v: torch.from_numpy(np.ascontiguousarray(v).reshape(-1)).cuda()
            rec["P"] = Problem(d, N, dev(a), dev(b))
            rec["f"] = dev(f)
        fb = lib().lgp_factor_bytes(rec["P"].handle, r["T"], r["T"], lgpcg.LGP_F64)
        rec["bytes"] = int(lib().lgp_problem_bytes(d, N) + fb + _vector_bytes(rec["P"].n))

    def _admit(self, rec):
        r = rec["req"]
        P = rec["P"]
        with torch.cuda.stream(self.stream):
            M = Factor(P, r["T"])
            F = P.load_vector(rec.pop("f"))
            x = torch.zeros_like(F)
        key = self._key(P, M)
        for B in self.batches[key]:
            slot, _, st = B.add(P, M, F, x, rtol=r["tol"], check=False)
            if st == "LGP_OK":
                break
            if st != "LGP_E_NOMEM":
                raise RuntimeError("lgp_batch_add: %s" % st)
        else:
            B = Batch(P, self.slots, stream=self.stream)
            self.batches[key].append(B)
            slot, _, st = B.add(P, M, F, x, rtol=r["tol"], check=False)
            if st != "LGP_OK":
                raise RuntimeError("lgp_batch_add: %s" % st)
        rec.update(batch=B, slot=slot, x=x, admit=time.perf_counter())
        del rec["P"]

    def serve(self, requests, arrivals):
        """Run `requests` (list of dicts) arriving at `arrivals` (seconds from
        the start, nondecreasing). Returns one record per request: arrival,
        admission and finish times (seconds from the start), latency, PCG
        iterations, true residual, status, and the solution (device)."""
        order = sorted(range(len(requests)), key=lambda i: arrivals[i])
        pending = collections.deque(order)
        recs = [dict(req=requests[i], arrival=float(arrivals[i])) for i in range(len(requests))]
        active = []
        t0 = time.perf_counter()
        while pending or active:
            now = time.perf_counter() - t0
            # admission, in arrival order, while the budget allows (a request
            # is admitted alone even when it exceeds the budget)
            while pending and recs[pending[0]]["arrival"] <= now:
                rec = recs[pending[0]]
                if "bytes" not in rec:
                    self._prepare(rec)
                if active and self.used + rec["bytes"] > self.budget:
                    break
                pending.popleft()
                self._admit(rec)
                self.used += rec["bytes"]
                active.append(rec)
                now = time.perf_counter() - t0
            if not active:
                if pending:
                    time.sleep(max(0.0, min(0.01, recs[pending[0]]["arrival"] - now)))
                continue
            # one round: every batch with running requests advances
            seen = set()
            for rec in active:
                B = rec["batch"]
                if id(B) in seen:
                    continue
                seen.add(id(B))
                B.step(self.step_iters)
            done = []
            for rec in active:
                info, fin = rec["batch"].info(rec["slot"])
                if fin:
                    rec["finish"] = time.perf_counter() - t0
                    rec["info"] = info
                    done.append(rec)
            for rec in done:
                active.remove(rec)
                rec["batch"].remove(rec["slot"])
                self.used -= rec["bytes"]
                rec["admit"] -= t0
                rec["latency"] = rec["finish"] - rec["arrival"]
                del rec["batch"]
            # batches with no request left are dropped (their workspace goes)
            for key in list(self.batches):
                self.batches[key] = [B for B in self.batches[key] if B.keep]
                if not self.batches[key]:
                    del self.batches[key]
        torch.cuda.synchronize()
        return recs


def poisson_arrivals(count: int, rate: float, seed: int = 4):
    """Arrival times of a Poisson stream of `rate` requests per second."""
    gaps = np.random.default_rng(seed).exponential(1.0 / rate, size=count)
    return np.cumsum(gaps) - gaps[0]


def latency_summary(recs):
    lat = np.array([r["latency"] for r in recs])
    span = max(r["finish"] for r in recs) - min(r["arrival"] for r in recs)
    return dict(requests=len(recs), p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                mean_s=float(lat.mean()), solves_per_sec=len(recs) / span, span_s=span,
                all_ok=all(r["info"]["status"] == "LGP_OK" for r in recs))
