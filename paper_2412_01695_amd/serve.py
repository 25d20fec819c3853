"""Continuous-batching solve server: many Davidson requests sharing one GPU.

Each request is one crystal (lattice, cutoff, k-point list, bands, atoms)
whose lowest bands are wanted at every k-point.  The server keeps a FIFO of
arrived requests and a fixed number of slots; a slot owns a HIP stream.
A request is admitted as soon as a slot is free *and* its device footprint
fits in what the HBM budget has left (the paper's "memgpu" input, Sec. 5.1,
sizes how many k-points are loaded at once; here it decides which requests
run side by side).  Admitted requests run concurrently on their own streams,
so their kernels overlap on the device; a request that finishes frees its
slot and memory and the next waiting request is admitted at once — the
batch changes continuously instead of being drained and refilled.
Converged wavefunctions stay resident on the device (an LRU store bounded
in bytes) for follow-up work such as a DFPT solve.

Per-request latency is completion minus arrival on the host monotonic clock.
The mixed-precision solve is the default (complex64 H|psi>, FP64 basis,
Rayleigh-Ritz and FP64 refinement to the tolerance).
"""
from __future__ import annotations

import argparse
import collections
import json
import math
import sys
import threading
import time

import numpy as np

from . import mkpw, synth

_VLOC_CACHE = {}
_VLOC_LOCK = threading.Lock()

def projector_table(cfg, npw, npwx, mall, kchunk=128):
    """beta_p(k+G) in the library's (nk, nproj, npwx) layout, zero padded, from
    the concatenated Miller indices of every k (library order), built in
    chunks of k-points (one vectorised evaluation per chunk, in the calling
    thread)."""
    beta = np.zeros((cfg.nk, cfg.nproj, npwx), dtype=np.complex128)
    off = np.concatenate([[0], np.cumsum(npw)]).astype(np.int64)
    b = synth.reciprocal_rows(cfg.lat)

    def chunk(k0):
        k1 = min(cfg.nk, k0 + kchunk)
        n = np.asarray(npw[k0:k1])
        kl = np.repeat(np.arange(k1 - k0), n)
        m = mall[off[k0]:off[k1]]
        q = cfg.kpts[k0:k1][kl] + m.astype(np.float64) @ b
        pos = np.arange(m.shape[0]) - np.repeat(off[k0:k1] - off[k0], n)
        beta[k0 + kl, :, pos] = synth.beta_values(cfg, q).T

    for k0 in range(0, cfg.nk, kchunk):
        chunk(k0)
    return beta


def _vloc(cfg):
    # V(r) depends on the mesh and the atoms only (the model potential's
    # Gaussian is negligible far inside any cutoff used here)
    key = (tuple(cfg.fft), len(cfg.tau))
    with _VLOC_LOCK:
        v = _VLOC_CACHE.get(key)
    if v is None:
        c = synth.Config(cfg.name, cfg.lat, 45.0, cfg.fft, cfg.kpts[:1], cfg.nbnd, cfg.tau, cfg.projectors,
                         cfg.dij, cfg.seed)
        v = synth.vloc_grid(c)
        with _VLOC_LOCK:
            _VLOC_CACHE[key] = v
    return v


def footprint_bytes(nk, npwx, nbnd, nproj, prec, basis_factor=4):
    """Device bytes a Davidson request holds: basis and H basis, Ritz and
    residual blocks, the caller's psi, projectors, reduced matrices, maps."""
    nbmax = min(basis_factor * nbnd, 64)
    c16 = 16
    b = 2 * nk * nbmax * npwx * c16                   # V, HV
    b += 5 * nk * nbnd * npwx * c16                   # X, HX, T, R, psi
    if prec == mkpw.PW_MIXED:
        b += 2 * nk * nbnd * npwx * 8                 # complex64 staging
    b += nk * nproj * npwx * (c16 + 8)                # beta (both precisions)
    b += nk * nbmax * (nbmax + 2 * nbnd) * c16        # H~, C, projections
    b += nk * npwx * (8 + 4 + 8)                      # kinetic, maps, H_diag
    return int(b * 1.05) + (4 << 20)


def npw_estimate(cfg):
    """Upper estimate of the sphere size (for admission before the basis is built)."""
    vol_sphere = 4.0 / 3.0 * math.pi * cfg.ecut_ry ** 1.5
    vol_cell = (2 * math.pi) ** 3 / cfg.omega
    n = vol_sphere / vol_cell
    return int(n + 4.0 * n ** (2.0 / 3.0) + 16)


class Request:
    def __init__(self, rid, arrival, cfg, tol_ry=1e-6, prec=mkpw.PW_MIXED, max_iter=300):
        self.id = rid
        self.arrival = arrival      # seconds on the server clock
        self.cfg = cfg
        self.tol_ry = tol_ry
        self.prec = prec
        self.max_iter = max_iter
        self.admitted = None
        self.done = None
        self.eig = None
        self.iters = None
        self.status = None
        self.error = None
        self.t_setup = self.t_solve = None   # host set-up (basis, maps, potential, projectors), device solve
        npwx = (npw_estimate(cfg) + 63) // 64 * 64
        self.bytes = footprint_bytes(cfg.nk, npwx, cfg.nbnd, cfg.nproj, prec)

    @property
    def latency(self):
        return None if self.done is None else self.done - self.arrival


class Server:
    def __init__(self, device=0, slots=8, hbm_budget_bytes=64 << 30, resident_bytes=8 << 30):
        import torch
        self.torch = torch
        self.device = device
        self.budget = int(hbm_budget_bytes)
        self.in_use = 0
        self.queue = collections.deque()
        self.cv = threading.Condition()
        self.stop = False
        self.t0 = time.monotonic()
        self.resident = collections.OrderedDict()   # id -> (eig, psi on device)
        self.resident_bytes = 0
        self.resident_cap = int(resident_bytes)
        self.completed = []
        self.streams = [torch.cuda.Stream(device=device) for _ in range(slots)]
        self.workers = [threading.Thread(target=self._worker, args=(i,), daemon=True) for i in range(slots)]
        for w in self.workers:
            w.start()

    def now(self):
        return time.monotonic() - self.t0

    def submit(self, req: Request):
        if req.bytes > self.budget:
            req.status = mkpw.PW_ENOMEM
            req.error = "request larger than the HBM budget"
            req.done = self.now()
            with self.cv:
                self.completed.append(req)
            return
        with self.cv:
            self.queue.append(req)
            self.cv.notify_all()

    def _take(self):
        # FIFO admission: the head waits until its footprint fits
        with self.cv:
            while True:
                if self.stop and not self.queue:
                    return None
                if self.queue and self.in_use + self.queue[0].bytes <= self.budget:
                    r = self.queue.popleft()
                    self.in_use += r.bytes
                    r.admitted = self.now()
                    return r
                self.cv.wait(0.05)

    def _release(self, r):
        with self.cv:
            self.in_use -= r.bytes
            self.completed.append(r)
            self.cv.notify_all()

    def _worker(self, slot):
        torch = self.torch
        stream = self.streams[slot]
        torch.cuda.set_device(self.device)
        while True:
            r = self._take()
            if r is None:
                return
            try:
                self._solve(r, stream)
            except Exception as e:  # a failed request does not take the server down
                r.status = -99
                r.error = repr(e)
            r.done = self.now()
            self._release(r)

    def _solve(self, r, stream):
        torch = self.torch
        cfg = r.cfg
        t0 = time.monotonic()
        ctx = mkpw.pw_create(self.device, stream.cuda_stream)
        try:
            mkpw.pw_set_lattice(ctx, cfg.lat)
            mkpw.pw_set_cutoff(ctx, cfg.ecut_ry, cfg.fft)
            npw, npwx = mkpw.pw_set_kpoints(ctx, cfg.kpts)
            mkpw.pw_set_vloc(ctx, _vloc(cfg))
            # projector values at every k+G of the library's order
            mall = mkpw.pw_get_miller_all(ctx, npw)
            mkpw.pw_set_projectors(ctx, projector_table(cfg, npw, npwx, mall), cfg.dij)
            t1 = time.monotonic()
            with torch.cuda.stream(stream):
                d_psi = torch.empty((cfg.nk, cfg.nbnd, npwx), dtype=torch.complex128, device=f"cuda:{self.device}")
                mkpw.pw_init_guess(ctx, cfg.nbnd, cfg.seed, d_psi)
                st, eig, iters, conv = mkpw.pw_davidson(ctx, r.prec, cfg.nbnd, d_psi, cfg.nk, r.tol_ry, r.max_iter)
                stream.synchronize()
            r.t_setup, r.t_solve = t1 - t0, time.monotonic() - t1
            r.status, r.eig, r.iters = st, eig, iters
            self._keep(r.id, eig, d_psi)
        finally:
            mkpw.pw_destroy(ctx)

    def _keep(self, rid, eig, d_psi):
        nbytes = d_psi.numel() * d_psi.element_size()
        with self.cv:
            self.resident[rid] = (eig, d_psi)
            self.resident_bytes += nbytes
            while self.resident_bytes > self.resident_cap and len(self.resident) > 1:
                _, (_, old) = self.resident.popitem(last=False)
                self.resident_bytes -= old.numel() * old.element_size()

    def warmup(self, reqs):
        """Solve `reqs` (all at once, no arrival times) and forget them: the
        H|psi> launch shapes the process tunes on first use for each precision,
        mesh, window and batch size are then in place before traffic arrives,
        as a server does at start-up."""
        for r in reqs:
            r.arrival = self.now()
            self.submit(r)
        while True:
            with self.cv:
                if len(self.completed) >= len(reqs):
                    self.completed.clear()
                    self.resident.clear()
                    self.resident_bytes = 0
                    return [r for r in reqs if r.status != 0]
            time.sleep(0.01)

    def close(self):
        with self.cv:
            self.stop = True
            self.cv.notify_all()
        for w in self.workers:
            w.join()


def prewarm(reqs):
    """Build the potential of every (mesh, atoms) pair the stream will use (one-off)."""
    for r in reqs:
        _vloc(r.cfg)


def replay(reqs, server: Server, speed=1.0, report=None):
    """Submit (arrival, Request) pairs at their arrival times; wait for all.
    `report(n)` is called after every 100th submission."""
    t_start = server.now()
    for i, r in enumerate(reqs):
        wait = t_start + r.arrival / speed - server.now()
        if wait > 0:
            time.sleep(wait)
        r.arrival = server.now()   # the moment it reached the server
        server.submit(r)
        if report and (i + 1) % 100 == 0:
            report(i + 1)
    while True:
        with server.cv:
            if len(server.completed) >= len(reqs):
                break
        time.sleep(0.01)


def summarize(reqs, wall):
    ok = [r for r in reqs if r.status == 0]
    lat = np.array([r.latency for r in ok])
    kb = sum(r.cfg.nk * r.cfg.nbnd for r in ok)

    def mean(v):
        return float(np.mean(v)) if len(v) else None
    return {"requests": len(reqs), "ok": int(lat.size),
            "mean_queue_s": mean([r.admitted - r.arrival for r in ok]),
            "mean_setup_s": mean([r.t_setup for r in ok]), "mean_solve_s": mean([r.t_solve for r in ok]),
            "p50_s": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_s": float(np.percentile(lat, 99)) if lat.size else None,
            "mean_s": float(lat.mean()) if lat.size else None,
            "throughput_req_s": lat.size / wall, "kband_solved_per_s": kb / wall, "wall_s": wall}


def make_requests(n, rate=20.0, seed=2024, tol_ry=1e-6, prec=mkpw.PW_MIXED):
    return [Request(i, t, cfg, tol_ry, prec) for i, (t, cfg) in enumerate(synth.serving_requests(n, rate, seed))]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=1000)
    ap.add_argument("--rate", type=float, default=20.0)
    ap.add_argument("--slots", type=int, default=8)
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--warmup", type=int, default=48, help="start-up requests (another seed) before the stream")
    args = ap.parse_args()

    def progress(msg):
        print(f"[serve {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)

    reqs = make_requests(args.requests, args.rate)
    prewarm(reqs)
    srv = Server(0, args.slots, int(args.budget_gb * (1 << 30)))
    bad = []
    if args.warmup > 0:
        # start-up: requests of the same distribution (another seed) tune the
        # H|psi> launch shapes before traffic arrives
        warm = make_requests(args.warmup, args.rate, seed=7)
        prewarm(warm)
        t = time.monotonic()
        bad = srv.warmup(warm)
        progress(f"start-up warm-up of {len(warm)} requests in {time.monotonic() - t:.1f} s"
                 f"{'' if not bad else f' ({len(bad)} failed)'}")
    t = time.monotonic()
    replay(reqs, srv, report=lambda n: progress(f"{n} requests submitted"))
    wall = time.monotonic() - t
    srv.close()
    out = summarize(reqs, wall)
    out["warmup_failed"] = len(bad)
    out["stream"] = (f"{args.requests} Poisson arrivals at {args.rate:g}/s: nk U{{16..1024}}, ecut U[20,45] Ry, "
                     f"nbnd U{{8..32}}, 1-2 atoms; mixed precision refined to 1e-6 Ry; {args.slots} slots, "
                     f"{args.budget_gb:g} GiB HBM budget; server warmed up with {args.warmup} requests of "
                     f"another seed (launch shapes tuned); one server process")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
