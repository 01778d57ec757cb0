"""Writes adjoint2d_fd.json: the loss, its central finite-difference
gradients (relative step 1e-6) and its complex-step gradients (exact to
round-off) for the 2D adjoint workload (256 x 256, 2000 steps), computed
with the FP64 CPU oracle only.

Loss: L = 1/2 sum (phi_T - phi_t)^2, phi_t the oracle's phi after the same
number of steps with delta = 0.025, tau = 1.2, g beta = 2e-5; parameters at
delta = 0.02, tau = 1.0, D = 1, g beta = 1e-5.

    python tests/golden/make_adjoint2d_fd.py [--steps 2000]
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import pyoracle  # noqa: E402
from paper_2608_26908_amd.workloads import workload  # noqa: E402


def with_param(cfg, name, value):
    c = dict(cfg)
    if name == "delta":
        c["delta"] = [[0, value], [value, 0]]
    elif name == "tau_pf":
        c["tau_pf"] = value
    elif name == "D":
        c["D"] = [[0.0], [value]]
    elif name == "gbeta":
        c["gbeta"] = [value]
    return c


def value(cfg, name):
    return {"delta": cfg["delta"][0][1], "tau_pf": cfg["tau_pf"], "D": cfg["D"][1][0],
            "gbeta": cfg["gbeta"][0]}[name]


def run(cfg, steps):
    s = pyoracle.OracleSim(cfg)
    s.step(steps)
    return s.get("phi")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--h", type=float, default=1e-6)
    args = ap.parse_args()
    cfg = workload("adjoint2d")
    tg = cfg["target"]
    tcfg = with_param(with_param(with_param(cfg, "delta", tg["delta"]), "tau_pf", tg["tau_pf"]),
                      "gbeta", tg["gbeta"])
    t0 = time.time()
    target = run(tcfg, args.steps)
    loss = 0.5 * float(((run(cfg, args.steps) - target) ** 2).sum())
    grads = {}
    for name in ("delta", "tau_pf", "D", "gbeta"):
        p = value(cfg, name)
        dp = args.h * abs(p)
        lp = 0.5 * float(((run(with_param(cfg, name, p + dp), args.steps) - target) ** 2).sum())
        lm = 0.5 * float(((run(with_param(cfg, name, p - dp), args.steps) - target) ** 2).sum())
        grads[name] = (lp - lm) / (2 * dp)
        print(name, grads[name], f"{time.time() - t0:.0f}s", flush=True)
    cs = {}
    base = pyoracle.OracleSim(cfg)
    for name in ("delta", "tau_pf", "D", "gbeta"):
        _, cs[name] = base.loss_grad_cs(args.steps, target, name)
        print("complex step", name, cs[name], f"{time.time() - t0:.0f}s", flush=True)
    out = {"workload": "adjoint2d", "steps": args.steps, "relative_step": args.h, "loss": loss,
           "grads": grads, "grads_complex_step": cs, "params": {k: value(cfg, k) for k in grads},
           "target_params": tg, "made_by": "tests/golden/make_adjoint2d_fd.py (FP64 oracle only)"}
    with open(os.path.join(HERE, "adjoint2d_fd.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
