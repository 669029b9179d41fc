"""The PAH-in-the-loop iteration (paper Sec. 2 with transiently heated PAHs):
a packet absorbed by a PAH leaves at a wavelength drawn from the cell's PAH
emission spectrum, which depends on the field the previous pass measured.

  pass 0 field: optically thin starlight at each leaf centre;
  repeat: PAH emission per cell (exact solver, or the surrogate with exact
  fallback) -> re-emission rows -> transport pass -> temperatures and mean
  intensity -> until the emitted PAH band power changes by less than tol.

Orchestration only; every numerical step is a libmcrt.so kernel.
"""
from __future__ import annotations

import numpy as np
import torch

from .mcrt import Engine, u64_view
from .pah import PahSolver


def relative_change(new, old):
    """Largest relative change of the band powers between two passes (the
    iteration's stop test; a few dozen numbers, on the host)."""
    a, b = new.cpu().numpy(), old.cpu().numpy()
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))


class PahLoop:
    def __init__(self, w, precision=None, surrogates=None, M=500):
        self.w = w
        self.eng = Engine.from_workload(w, precision=precision)
        self.eng.build_tables(w.source.pos, w.source.lum, w.source.teff)
        self.solvers = [PahSolver.from_model(pm, M=M) for pm in w.pah]
        self.surrogates = surrogates or [None] * len(self.solvers)
        dev = self.eng.device
        self.rows = torch.empty((len(self.solvers), self.eng.n_cells, self.eng.n_lambda),
                                dtype=torch.float64, device=dev)
        self.mass = self.eng.cell_mass()

    def emission(self, J):
        outs = []
        for p, (s, sur) in enumerate(zip(self.solvers, self.surrogates)):
            if sur is not None:
                out = sur.solve(J)[0]
            else:
                out = s.solve(J)[0]
            s.rows(out, rows=self.rows[p])
            outs.append(out)
        return outs

    def run(self, n_iter=4, n_packets=None, seed=None, tol=0.01, log=None, batch=None):
        """batch: packets per transport call (id ranges that fit the deferred
        tally's workspace, when one is set on the engine); None = one call."""
        w = self.w
        N = int(n_packets or w.n_packets)
        seed = w.seed if seed is None else seed
        J = self.eng.thin_field()
        hist = []
        prev = None
        res = {}
        for it in range(n_iter):
            outs = self.emission(J)
            tal = self.eng.new_tallies(tally_j=True)
            self.eng.run_batched(tal, 0, N, N, seed + 7919 * it, batch or N, pah_rows=self.rows)
            T = self.eng.temperatures(tal["nabs"], N)
            J = self.eng.mean_intensity(tal["jq"], N)
            bp = torch.stack([s.band_power(o, self.mass) for s, o in zip(self.solvers, outs)])
            change = None if prev is None else relative_change(bp, prev)
            prev = bp
            cnt = u64_view(tal["counters"])
            hist.append(dict(iteration=it, change=change, pah_abs=int(cnt[9]), escaped=int(cnt[1])))
            if log:
                log(hist[-1])
            res = dict(tallies=tal, T=T, J=J, outs=outs, history=hist)
            if change is not None and change < tol:
                break
        return res
