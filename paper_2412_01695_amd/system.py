"""Load a synthetic crystal into a library context (host-side marshalling).

``System(cfg)`` creates a ``pw_ctx`` for one ``synth.Config``: lattice,
cutoff and FFT mesh, the k-point list (the library builds the bases), the
local potential on the mesh, the projector values at every k+G of the
library's own plane-wave order and, when the config has them, the overlap
coefficients q.  It also lays out wavefunction arrays in
the library's (nk, nvec, npwx) format.
"""
from __future__ import annotations

import numpy as np

from . import mkpw, synth


class System:
    def __init__(self, cfg: synth.Config, device: int = 0, stream=None, vloc=None, with_projectors=True,
                 dij=None):
        self.cfg = cfg
        self.device = device
        self.stream = None
        ptr = None
        if device >= 0:
            import torch
            # the context orders its work on this torch stream (default priority);
            # torch's default stream has handle 0, which the C-ABI reads as "no stream"
            if stream is None:
                self.stream = torch.cuda.Stream(device=device)
            elif isinstance(stream, torch.cuda.Stream):
                self.stream = stream
            else:
                self.stream = torch.cuda.ExternalStream(int(stream), device=device) if stream else \
                    torch.cuda.Stream(device=device)
            ptr = self.stream.cuda_stream
        self.ctx = mkpw.pw_create(device, ptr)
        try:
            mkpw.pw_set_lattice(self.ctx, cfg.lat)
            mkpw.pw_set_cutoff(self.ctx, cfg.ecut_ry, cfg.fft)
            self.npw, self.npwx = mkpw.pw_set_kpoints(self.ctx, cfg.kpts)
            self.miller = [mkpw.pw_get_miller(self.ctx, ik, int(n)) for ik, n in enumerate(self.npw)]
            if device >= 0 or vloc is not None:
                self.vloc = synth.vloc_grid(cfg) if vloc is None else np.asarray(vloc, dtype=np.float64)
                mkpw.pw_set_vloc(self.ctx, self.vloc)
            if with_projectors and cfg.nproj > 0:
                beta = np.zeros((cfg.nk, cfg.nproj, self.npwx), dtype=np.complex128)
                q = np.concatenate([synth.q_vectors(cfg, ik, m) for ik, m in enumerate(self.miller)])
                ball = synth.beta_values(cfg, q)
                o = 0
                for ik in range(cfg.nk):
                    n = int(self.npw[ik])
                    beta[ik, :, :n] = ball[:, o:o + n]
                    o += n
                self.beta = beta
                mkpw.pw_set_projectors(self.ctx, beta, cfg.dij if dij is None else dij)
                if cfg.qij is not None:
                    mkpw.pw_set_qij(self.ctx, cfg.qij)
        except Exception:
            mkpw.pw_destroy(self.ctx)
            self.ctx = None
            raise

    @property
    def nk(self) -> int:
        return self.cfg.nk

    def close(self):
        if self.ctx is not None:
            mkpw.pw_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def layout(self, rows_by_k, nvec: int | None = None) -> np.ndarray:
        """Pack per-k (nvec, npw_k) arrays into the (nk, nvec, npwx) complex128 layout."""
        nvec = rows_by_k[0].shape[0] if nvec is None else nvec
        out = np.zeros((self.nk, nvec, self.npwx), dtype=np.complex128)
        for ik, r in enumerate(rows_by_k):
            out[ik, :r.shape[0], :self.npw[ik]] = r
        return out

    def unpack(self, arr) -> list:
        """(nk, nvec, npwx) -> list of (nvec, npw_k) arrays."""
        a = np.asarray(arr)
        return [a[ik, :, :self.npw[ik]] for ik in range(self.nk)]

    def psi_guess(self, nbnd: int | None = None, seed: int | None = None) -> np.ndarray:
        return synth.psi_guess_all(self.cfg, self.miller, self.npwx, nbnd, seed)
