"""KL divergence against the conditioning size (Eq. (9), Sec. V-B), on the GPU.

    python -m paper_2403_07412_amd.kl_curve --n 180000 --range 0.3

For each smoothness the Matern range beta comes from Table II (its value for
the effective range asked for), the points are uniform on the unit square
(seeded), and for each ordering the exact log-likelihood at y = 0 is
computed once by the dense Cholesky, then the Vecchia log-likelihood at y = 0
for every m.  One JSON line per (nu, ordering) goes to stdout.  The dense
factor takes 8 n^2 bytes of device memory (259 GB at n = 180,000).
"""
import argparse
import json
import sys
import time

import numpy as np
import torch

from . import VecchiaError, VecchiaNumericalError, kl_curve

# Table II: beta for effective range 0.1, 0.3, 0.8 at nu = 0.5, 1.5, 2.5 (the
# (0.3, 2.5) entry as given in the captions of Figs. 5 and 6)
TABLE2_BETA = {
    0.1: {0.5: 0.026270, 1.5: 0.017512, 2.5: 0.014290},
    0.3: {0.5: 0.078809, 1.5: 0.052537, 2.5: 0.042869},
    0.8: {0.5: 0.210158, 1.5: 0.140098, 2.5: 0.114318},
}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--n", type=int, default=20000)
    ap.add_argument("--range", type=float, default=0.3, choices=sorted(TABLE2_BETA))
    ap.add_argument("--nu", type=float, nargs="+", default=[0.5, 1.5, 2.5])
    ap.add_argument("--m", type=int, nargs="+", default=[10, 30, 60, 90, 120, 150])
    ap.add_argument("--orderings", nargs="+", default=["random", "morton"])
    ap.add_argument("--tau2", type=float, default=0.0)
    ap.add_argument("--seed", type=int, default=2024)
    args = ap.parse_args(argv)
    if not torch.cuda.is_available():
        print("kl_curve needs a GPU", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    free, total = torch.cuda.mem_get_info(dev)
    need = 8 * args.n * args.n
    if need > free:
        print(f"the dense factor needs {need / 1e9:.1f} GB, {free / 1e9:.1f} GB free", file=sys.stderr)
        return 1
    rng = np.random.default_rng(args.seed)
    locs = torch.from_numpy(rng.uniform(0.0, 1.0, size=(args.n, 2))).to(dev)
    for nu in args.nu:
        beta = TABLE2_BETA[args.range][nu]
        theta = torch.tensor([1.0, beta, args.tau2], dtype=torch.float64, device=dev)
        for ordering in args.orderings:
            t0 = time.perf_counter()
            rec = {"n": args.n, "nu": nu, "beta": beta, "tau2": args.tau2, "effective_range": args.range}
            try:
                rec.update(kl_curve(locs, args.m, nu, theta, ordering=ordering, seed=args.seed))
            except (VecchiaError, VecchiaNumericalError) as e:
                rec.update({"ordering": ordering, "error": str(e)})
            torch.cuda.synchronize()
            rec["seconds"] = round(time.perf_counter() - t0, 2)
            print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
