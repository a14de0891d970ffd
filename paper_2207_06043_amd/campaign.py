"""The paper's campaign observables on a running lattice (section
"Transport of an elastic capsule in a microfluidic bifurcation" and the
multiple-capsule section): the relative surface strain dS = S/S0 - 1 of
every body, its centre, Taylor deformation and largest link stretch,
recorded every K steps against the dimensionless time t u_max / d; the run
ends where the library stops it (a membrane link at twice its rest length,
or an unstable flow).  The surfaces, volumes and stretches come from the
library's diagnostics (lbm_diagnostics) and the positions from
lbm_get_body; this module only records them."""
from __future__ import annotations

import numpy as np

from ._abi import LBM_E_DAMAGED, LBM_E_UNSTABLE, LBM_OK

STATUS = {LBM_OK: "ok", LBM_E_DAMAGED: "damaged", LBM_E_UNSTABLE: "unstable"}


def taylor_deformation(x):
    """(sqrt(l1) - sqrt(l3)) / (sqrt(l1) + sqrt(l3)) of the second-moment
    tensor of the vertex positions x [nv, 3] about their mean."""
    d = x - x.mean(0)
    lam = np.linalg.eigvalsh(d.T @ d / len(x))
    a, c = np.sqrt(max(lam[2], 0.0)), np.sqrt(max(lam[0], 0.0))
    return float((a - c) / (a + c)) if a + c > 0 else 0.0


def log_run(lat, n_steps, every, u_max, d):
    """Advance lat by up to n_steps steps, recording every `every` steps.
    Returns {"t": [t u_max / d], "step": [...], "bodies": [{"dS": [...],
    "centre": [[x, y, z], ...], "taylor": [...], "stretch": [...],
    "peak_dS": ..., "t_peak": ...}], "status": "ok" | "damaged" |
    "unstable", "steps_done": ...}; the first record is the state at the
    start (dS = 0)."""
    diag0 = lat.diagnostics()
    S0 = [b[1] for b in diag0["bodies"]]
    nb = len(S0)
    step0 = lat.info()["steps_done"]
    log = {"t": [], "step": [], "bodies": [{"dS": [], "centre": [], "taylor": [], "stretch": []}
                                           for _ in range(nb)]}

    def record(diag, steps):
        log["step"].append(int(steps - step0))
        log["t"].append((steps - step0) * u_max / d)
        for b in range(nb):
            x = lat.body(b)[0].cpu().numpy()
            rec = log["bodies"][b]
            rec["dS"].append(diag["bodies"][b][1] / S0[b] - 1.0)
            rec["centre"].append([float(v) for v in x.mean(0)])
            rec["taylor"].append(taylor_deformation(x))
            rec["stretch"].append(diag["bodies"][b][2])

    record(diag0, step0)
    status, done = LBM_OK, 0
    while done < n_steps and status == LBM_OK:
        k = min(every, n_steps - done)
        lat.step(k)
        status = lat.sync(raise_on_stop=False)
        steps = lat.info()["steps_done"]
        done = steps - step0
        record(lat.diagnostics(), steps)
    for rec in log["bodies"]:
        k = int(np.argmax(rec["dS"]))
        rec["peak_dS"], rec["t_peak"] = rec["dS"][k], log["t"][k]
    log["status"] = STATUS.get(status, str(status))
    log["steps_done"] = int(done)
    return log
