"""Central-difference check of the autograd gradient at full size.

``python -m paper_1804_01184_amd.fdcheck`` builds the 1001² smooth benchmark (1001² + 40 PML,
64 shots, 4000 steps, smooth random Vp with Gardner density and 8 Gaussian
anomalies), takes the gradient of J = ½‖d(m) − d_obs‖² through
FWIFunction (forward with checkpoints every ⌈√nt⌉ steps, backward with
segment recompute), and compares ⟨∇J, δm⟩ with (J(m + hδm) − J(m − hδm))/2h
along seeded smooth random directions δm (zero within 5 cells of every
source; relative to the model), for h in {1e-2, 3e-3, 1e-3, 3e-4, 1e-4}.  J of the
differences is summed in FP64 from the FP32 traces.  Prints one JSON line
with the relative error of each direction at its best h.
"""
from __future__ import annotations

import json
import sys
import time

import numpy as np
import torch

from . import api, autograd, workloads as W


# central differences converge as h^2 until FP32 rounding of the traces
# takes over; the scan reaches below 1e-3, where the truncation error of the
# smoothest directions is still above 1e-3 on the 1001² smooth benchmark
HS = (1e-2, 3e-3, 1e-3, 3e-4, 1e-4)


def directions(w, n, seed=1804 + 30):
    rng = np.random.default_rng(seed)
    keep = np.ones((w.nz, w.nx))
    zz, xx = np.mgrid[0:w.nz, 0:w.nx]
    for x, z in w.src_xz.reshape(-1, 2):
        keep[(zz - z / w.dz) ** 2 + (xx - x / w.dx) ** 2 <= 25.0] = 0.0
    for _ in range(n):
        a = (W.smooth_noise(rng, w.nz, w.nx, 20.0) - 0.5) * keep
        b = (W.smooth_noise(rng, w.nz, w.nx, 20.0) - 0.5) * keep
        yield a, b


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="smooth1001", choices=["gauss401", "smooth1001"])
    ap.add_argument("--directions", type=int, default=16)
    ap.add_argument("--param", default="vp-rho")
    a = ap.parse_args(argv)
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    w = W.smooth1001() if a.workload == "smooth1001" else W.gauss401()
    k = int(np.ceil(np.sqrt(w.nt)))
    plan = api.Plan(api.Grid.of(w), w.src_xz, w.rec_xz, ckpt_every=k)
    f = torch.tensor(w.wavelet(), dtype=torch.float32, device=dev)
    obs = plan.forward("vp-rho", w.vp_true, w.rho_true, f)
    K0 = w.rho_start * w.vp_start ** 2
    m1n, m2n = (x.cpu().numpy() for x in api.model_convert(
        "k-rho", a.param, torch.tensor(K0, dtype=torch.float32, device=dev),
        torch.tensor(w.rho_start, dtype=torch.float32, device=dev)))
    m1 = torch.tensor(m1n, device=dev, requires_grad=True)
    m2 = torch.tensor(m2n, device=dev, requires_grad=True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    tr = autograd.model_traces(plan, a.param, m1, m2, f)
    (0.5 * ((tr - obs) ** 2).sum()).backward()
    torch.cuda.synchronize()
    t_grad = time.perf_counter() - t
    print(f"gradient through FWIFunction: {t_grad:.1f} s", file=sys.stderr, flush=True)
    del tr

    def J(x1, x2):
        d = plan.forward(a.param, x1, x2, f)
        return float(0.5 * ((d.double() - obs.double()) ** 2).sum())

    out = []
    t = time.perf_counter()
    for d1n, d2n in directions(w, a.directions):
        d1 = torch.tensor(d1n * m1n, dtype=torch.float32, device=dev)
        d2 = torch.tensor(d2n * m2n, dtype=torch.float32, device=dev)
        an = float((m1.grad.double() * d1.double()).sum() + (m2.grad.double() * d2.double()).sum())
        errs = {}
        for h in HS:
            fd = (J(m1.detach() + h * d1, m2.detach() + h * d2) -
                  J(m1.detach() - h * d1, m2.detach() - h * d2)) / (2 * h)
            errs[h] = abs(fd - an) / max(abs(an), 1e-300)
        hb = min(errs, key=errs.get)
        out.append({"analytic": an, "best_h": hb, "rel_err": errs[hb],
                    "rel_err_by_h": {str(h): e for h, e in errs.items()}})
        print(f"direction {len(out)}: rel err {errs[hb]:.2e} at h = {hb}", file=sys.stderr,
              flush=True)
    t_fd = time.perf_counter() - t
    info = plan.info
    print(json.dumps({"workload": w.name, "param": a.param, "padded": [info["Nz"], info["Nx"]],
                      "shots": w.nshots, "nt": w.nt, "ckpt_every": info["ckpt_every"],
                      "segments": info["segments"], "gradient_seconds": round(t_grad, 3),
                      "fd_seconds": round(t_fd, 1),
                      "max_rel_err": max(r["rel_err"] for r in out), "directions": out}),
          flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
