"""Estimation and prediction against the conditioning size on a synthetic field (the study of Sec. V-C).

    python -m paper_2403_07412_amd.kriging_study --n 20000 --test 2000

The paper fits the power-exponential model on great-circle distances to
soil-moisture and wind-speed residuals (250K training / 25K test points)
and compares the kriging MSE of the Vecchia fits with exact kriging.  Those
data are not available; this study draws a field of the same model exactly
(dense Cholesky of its covariance, torch on the GPU) on (longitude,
latitude) points over a 10 x 10 degree box.  Then, for each m, it runs:
  - random ordering and great-circle conditioning sets (vecchia_knn);
  - the maximum-likelihood fit at the true alpha (vecchia_mle, cov model);
  - conditioning sets of the test points among the training points
    (vecchia_knn_query);
  - kriging (vecchia_predict) and its mean squared error.
A dense kriging with the true parameters gives the reference MSE.  One
JSON line per m, then one for the reference, go to stdout.
"""
import argparse
import json
import sys
import time

import numpy as np
import torch

from . import GREAT_CIRCLE, POWEXP, vecchia_knn, vecchia_knn_query, vecchia_mle, vecchia_predict

EARTH_RADIUS_KM = 6371.0


def great_circle_km(a, b):
    """Pairwise great-circle distances (haversine, differences in degrees first) of two (lon, lat) sets."""
    d2r = np.pi / 180.0
    lat_a, lat_b = a[:, 1:2] * d2r, b[None, :, 1] * d2r
    s1 = torch.sin(0.5 * (a[:, 1:2] - b[None, :, 1]) * d2r)
    s2 = torch.sin(0.5 * (a[:, 0:1] - b[None, :, 0]) * d2r)
    h = torch.clamp(s1 * s1 + torch.cos(lat_a) * torch.cos(lat_b) * s2 * s2, max=1.0)
    return 2.0 * EARTH_RADIUS_KM * torch.asin(torch.sqrt(h))


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--n", type=int, default=20000, help="training points")
    ap.add_argument("--test", type=int, default=2000, help="test points")
    ap.add_argument("--m", type=int, nargs="+", default=[10, 30, 60, 90, 120, 150])
    ap.add_argument("--alpha", type=float, default=0.9)
    ap.add_argument("--theta", type=float, nargs=3, default=[1.0, 60.0, 0.05], metavar=("SIGMA2", "BETA", "TAU2"))
    ap.add_argument("--seed", type=int, default=2403)
    args = ap.parse_args(argv)
    if not torch.cuda.is_available():
        print("kriging_study needs a GPU", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(args.seed)
    nt = args.n + args.test
    pts = np.column_stack([rng.uniform(-95.0, -85.0, nt), rng.uniform(30.0, 40.0, nt)])
    P = torch.from_numpy(pts).to(dev)
    s2, beta, tau2 = args.theta
    # exact draw of the whole field: Sigma = s2 exp(-d^alpha / beta) + tau2 I
    t0 = time.perf_counter()
    S = great_circle_km(P, P)
    S.pow_(args.alpha).div_(-beta).exp_().mul_(s2)
    S.diagonal().add_(tau2)
    Lc = torch.linalg.cholesky(S)
    y = Lc @ torch.from_numpy(rng.standard_normal(nt)).to(dev)
    del Lc
    perm = torch.from_numpy(rng.permutation(nt)).to(dev)
    train, test = perm[: args.n], perm[args.n:]
    # exact kriging with the true parameters (the reference)
    Stt = S[train][:, train]
    Sqt = S[test][:, train]
    mean_exact = Sqt @ torch.linalg.solve(Stt, y[train])
    mse_exact = float(((mean_exact - y[test]) ** 2).mean())
    del S, Stt, Sqt
    torch.cuda.empty_cache()
    draw_s = time.perf_counter() - t0
    Ltr = P[train].contiguous()          # random ordering: the permutation above
    ytr = y[train].contiguous()
    Lte = P[test].contiguous()
    yte = y[test]
    cov = (POWEXP, GREAT_CIRCLE, args.alpha)
    theta0 = (0.5 * s2, 0.5 * beta, 2.0 * tau2 + 1e-3)
    for m in args.m:
        t1 = time.perf_counter()
        nbr = vecchia_knn(Ltr, m, metric=GREAT_CIRCLE)
        fit = vecchia_mle(Ltr, ytr, nbr, m, 0.0, theta0, cov=cov)
        qn = vecchia_knn_query(Ltr, Lte, m, metric=GREAT_CIRCLE)
        th = torch.tensor(fit["theta"], dtype=torch.float64, device=dev)
        mean, var, st = vecchia_predict(Ltr, ytr, Lte, qn, m, cov, th)
        mse = float(((mean - yte) ** 2).mean())
        torch.cuda.synchronize()
        print(json.dumps({"m": m, "theta_hat": [float(x) for x in fit["theta"]], "loglik": fit["loglik"],
                          "iterations": fit["iterations"], "evaluations": fit["evaluations"], "mse": mse,
                          "status": int(st.item()), "seconds": round(time.perf_counter() - t1, 3)}), flush=True)
    print(json.dumps({"reference": "exact kriging, true parameters", "mse": mse_exact, "n_train": args.n,
                      "n_test": args.test, "theta_true": [s2, beta, tau2], "alpha": args.alpha,
                      "draw_and_reference_seconds": round(draw_s, 2)}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
