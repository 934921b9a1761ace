"""Poisson-arrival driver of the serving core (nao_server) and its latency report.

Requests are SCF-iteration pairs (density update from a fresh density matrix, then the
Hamiltonian with the structure's potential) for structures of 20-400 atoms shaped like the
100-atom block or the 375-atom slab.  Sessions keep a structure resident for 10-40
iterations; a request joins the oldest session with no request in flight, otherwise it opens
a new session.  The structures come from a pool generated before the run.  Every iteration
has a fresh density matrix D = C C^T (C seeded per session and iteration), built on the
device by a staging thread while the session's previous iteration runs; the staging time and
the driver's waits for it are reported separately.

Two paths are compared:
  * plain:   FP64, one request per launch, one slot, every octree batch its own unit;
  * batched: a reduced precision (FP32 by default: within 1e-6 of FP64 and the fastest form on
             this GPU; bf16x6 meets the same bound), several requests per launch, several
             slots, execution groups of up to 256 points.
"""
from __future__ import annotations

import math
import time

import numpy as np

from workloads import generate as g


def make_pool(n_structures, seed=0, min_atoms=20, max_atoms=400, grid_scale=1.0):
    """Structures drawn log-uniformly in size, style 2 (block) or 4 (slab) by a coin flip; with
    three or more structures the first two are the smallest and the largest size, so that the
    pool spans the whole range."""
    rng = g.rng_for(5, seed, g.STREAM_ARRIVAL)
    pool = []
    for k in range(n_structures):
        n = int(round(math.exp(rng.uniform(math.log(min_atoms), math.log(max_atoms)))))
        if n_structures >= 3 and k < 2:
            n = (min_atoms, max_atoms)[k]
        style = 2 if rng.uniform() < 0.5 else 4
        xyz = g.serving_geometry(style, n, 1000 * seed + k)
        p = dict(g.CONFIGS[style])
        if grid_scale != 1.0:
            p["n_r"] = max(8, int(p["n_r"] * grid_scale))
            p["n_ang"] = max(14, int(p["n_ang"] * grid_scale))
        w = g.make_workload(xyz, p, 5, 1000 * seed + k, with_density=False)
        w["style"] = style
        w["d_max"] = p["d_max"]
        w["n_occ"] = 2 * len(xyz)
        pool.append(w)
    return pool


def measure_pool(nao, pool):
    """Work measure U = sum_b |B_b| m_b^2 of every pool structure (both operations use the same
    batches), stored as w["units"]."""
    home = nao.Context(0)
    for w in pool:
        s = nao.build_batches(home, w["basis"], w["xyz"], w["w"], w["max_batch"])
        w["units"] = s.work_units()
        s.close()
    home.close()


class DensityStager:
    """Fresh seeded D = C C^T per (session, iteration), built on the GPU with torch and zeroed
    between centres farther apart than d_max (input staging, not part of the method).

    A worker thread prepares iteration k + 1 of a session while iteration k runs, on a stream
    of its own, so that the driver's loop neither waits for the GEMM nor for the server's work.
    """

    def __init__(self, torch, device):
        import queue
        import threading
        self.torch = torch
        self.device = device
        self.masks = {}
        self.stream = torch.cuda.Stream(device=device)
        self.jobs = queue.Queue()
        self.ready = {}                 # (session seed, iteration) -> D
        self.cv = threading.Condition()
        self.busy_s = 0.0
        self.worker = threading.Thread(target=self._run, daemon=True)
        self.worker.start()

    def upload(self, a):
        with self.torch.cuda.stream(self.stream):
            t = self.torch.from_numpy(a).to(self.device, non_blocking=False)
        self.stream.synchronize()
        return t

    def _make(self, work, session_seed, iteration):
        torch = self.torch
        key = id(work)
        if key not in self.masks:
            ba = g.basis_atom_index(work["basis"])
            xyz = work["basis"]["atom_xyz"]
            dd = np.sqrt(((xyz[:, None] - xyz[None]) ** 2).sum(-1))
            keep = (dd <= work["d_max"])[ba][:, ba]
            self.masks[key] = self.upload(keep)
        gen = torch.Generator(device=self.device)
        gen.manual_seed(int(session_seed) * 100003 + int(iteration))
        with torch.cuda.stream(self.stream):
            C = torch.randn((work["n_basis"], work["n_occ"]), generator=gen, dtype=torch.float64, device=self.device)
            D = C @ C.T
            D = 0.5 * (D + D.T)
            D.mul_(self.masks[key])
            D = D.contiguous()
        self.stream.synchronize()
        return D

    def _run(self):
        while True:
            job = self.jobs.get()
            if job is None:
                return
            work, seed, k = job
            t0 = time.perf_counter()
            D = self._make(work, seed, k)
            self.busy_s += time.perf_counter() - t0
            with self.cv:
                self.ready[(seed, k)] = D
                self.cv.notify_all()

    def request(self, work, seed, k):
        """Ask for iteration k of a session (returns at once)."""
        self.jobs.put((work, seed, k))

    def take(self, seed, k):
        """The D of iteration k (waits for the worker if it is not ready yet)."""
        with self.cv:
            while (seed, k) not in self.ready:
                self.cv.wait()
            return self.ready.pop((seed, k))

    def close(self):
        self.jobs.put(None)
        self.worker.join()
        self.ready.clear()


def run(nao, torch, pool, lam, duration_s, max_requests, path, precision="fp32", n_slots=3,
        max_per_launch=8, hbm_budget=0, seed=0, log=None, max_sessions=24):
    """One serving run; returns a dict with latency percentiles and throughput.  Latency runs
    from a request's arrival to its results being complete on the device: the driver's delay
    before the submit (waiting for a session, a staged D) plus the server's submit-to-done time.
    At most max_sessions sessions are open at once: an arrival that finds every open session busy
    and the limit reached waits in the driver's queue (a saturated path would otherwise open a
    session, and stage its next D, for every arrival)."""
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(np.random.SeedSequence([5, seed, g.STREAM_ARRIVAL, int(lam * 1000)]))
    home = nao.Context(0, hbm_budget=hbm_budget)
    if path == "plain":
        srv = nao.Server(home, n_slots=1, max_per_launch=1, precision="fp64", group_max=0)
    else:
        srv = nao.Server(home, n_slots=n_slots, max_per_launch=max_per_launch, precision=precision)
    stager = DensityStager(torch, dev)
    sessions = []  # dicts: sid, work, k, K, busy, seed
    tickets = {}   # ticket -> (session dict, D, delay before submit)
    lat, units_done, wait_s = [], 0.0, 0.0
    done = 0
    submitted = 0
    t0 = time.perf_counter()
    next_arrival = t0 + rng.exponential(1.0 / lam)
    vbuf = {}
    queue = []          # arrival times waiting for a session
    open_now, max_queue = 0, 0
    while True:
        now = time.perf_counter()
        if now - t0 > duration_s or done >= max_requests:
            break
        while now >= next_arrival and submitted + len(queue) < max_requests:
            queue.append(next_arrival)
            next_arrival += rng.exponential(1.0 / lam)
        max_queue = max(max_queue, len(queue))
        while queue:
            free = [s for s in sessions if not s["busy"] and s["k"] < s["K"]]
            if not free and open_now >= max_sessions:
                break
            arrival = queue.pop(0)
            if free:
                s = min(free, key=lambda x: x["opened"])
            else:
                open_now += 1
                w = pool[int(rng.integers(len(pool)))]
                sid = srv.open_session(w["basis"], w["xyz"], w["w"], w["max_batch"])
                s = dict(sid=sid, work=w, k=0, K=int(rng.integers(10, 41)), busy=False, opened=now,
                         seed=len(sessions) + 1)
                sessions.append(s)
                stager.request(w, s["seed"], 0)
            ts = time.perf_counter()
            D = stager.take(s["seed"], s["k"])
            v = None
            if s["k"] == 0:
                v = stager.upload(s["work"]["v"])
                vbuf[s["sid"]] = v
            wait_s += time.perf_counter() - ts
            if s["k"] + 1 < s["K"]:
                stager.request(s["work"], s["seed"], s["k"] + 1)
            tk = srv.submit(s["sid"], D, v)
            tickets[tk] = (s, D, time.perf_counter() - arrival)
            s["busy"] = True
            s["k"] += 1
            submitted += 1
        srv.step()
        for tk in list(tickets):
            st, t_sub, t_start, t_end = srv.poll(tk)
            if st == nao.REQ_FAILED:
                raise RuntimeError("request %d failed: %s" % (tk, home.last_error()))
            if st == nao.REQ_DONE:
                s, _, delay = tickets.pop(tk)
                s["busy"] = False
                lat.append(delay + (t_end - t_sub))
                done += 1
                units_done += s["work"].get("units", 0.0)
                if s["k"] >= s["K"]:
                    srv.close_session(s["sid"])
                    vbuf.pop(s["sid"], None)
                    open_now -= 1
        time.sleep(0.0002)
    elapsed = time.perf_counter() - t0
    # requests still waiting are dropped with the server; wait only for the running ones
    backlog = sum(1 for tk in tickets if srv.poll(tk)[0] == nao.REQ_WAITING)
    t_drain = time.perf_counter()
    while time.perf_counter() - t_drain < 120:
        running, _ = srv.step()
        if running == 0:
            break
        time.sleep(0.001)
    srv.close()
    home.close()
    stager.close()
    lat = np.array(lat) * 1e3
    out = dict(path=path, precision="fp64" if path == "plain" else precision, lam=lam,
               completed=int(done), submitted=int(submitted), seconds=round(elapsed, 2),
               requests_per_s=round(done / elapsed, 3),
               gpt_basis2_per_s=round(2.0 * units_done / elapsed / 1e9, 3),
               p50_ms=round(float(np.percentile(lat, 50)), 2) if len(lat) else None,
               p99_ms=round(float(np.percentile(lat, 99)), 2) if len(lat) else None,
               staging_busy_s=round(stager.busy_s, 2), staging_wait_s=round(wait_s, 2),
               sessions=len(sessions), backlog_at_end=int(backlog) + len(queue),
               driver_queue_max=int(max_queue))
    if log:
        log("serve %s" % out)
    return out


def main(argv=None):
    """python -m paper_1912_06636_amd.serve: one JSON line per (path, arrival rate)."""
    import argparse
    import json
    import sys

    import torch

    from paper_1912_06636_amd import nao

    ap = argparse.ArgumentParser()
    ap.add_argument("--lam", type=float, nargs="+", default=[2.0, 8.0, 32.0])
    ap.add_argument("--seconds", type=float, default=30.0)
    ap.add_argument("--max-requests", type=int, default=500)
    ap.add_argument("--paths", nargs="+", default=["plain", "batched"])
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--pool", type=int, default=6)
    ap.add_argument("--grid-scale", type=float, default=1.0)
    # sessions beyond the budget wait for releases (admission by footprint); a saturated path
    # would otherwise open sessions until the device runs out of memory
    ap.add_argument("--hbm-budget-gb", type=float, default=160.0)
    ap.add_argument("--slots", type=int, default=3)
    ap.add_argument("--max-per-launch", type=int, default=8)
    args = ap.parse_args(argv)

    def log(msg):
        print("[serve]", msg, file=sys.stderr, flush=True)

    t0 = time.time()
    pool = make_pool(args.pool, grid_scale=args.grid_scale)
    measure_pool(nao, pool)
    log("pool of %d structures (%s atoms) ready in %.1f s" % (
        len(pool), [len(w["basis"]["atom_xyz"]) for w in pool], time.time() - t0))
    for path in args.paths:
        for lam in args.lam:
            out = run(nao, torch, pool, lam, args.seconds, args.max_requests, path, precision=args.precision,
                      n_slots=args.slots, max_per_launch=args.max_per_launch,
                      hbm_budget=int(args.hbm_budget_gb * (1 << 30)), log=log)
            print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
