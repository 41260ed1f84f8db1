"""Train the learned boundary-cell correction and judge it against the plain smoother.

    python -m paper_2506_12899_amd.train_learned --out weights.bin [--geometries 200] [--n 16]

1. data: seeded training geometries (spheres / ellipsoids, p = 3, 3D), pairs
   from the method's own finest-level smoothing (see learned.py);
2. training: FP32 forward / loss / backward / Adam kernels of the library;
3. judge: GMRES iterations to 1e-8 with and without the correction on held-out
   geometries; the plain smoother stays the default where it is not beaten.

Writes the checkpoint and prints one JSON line with the loss history and the
A/B iteration counts.
"""
import argparse
import json
import sys
import time

import torch

from . import learned, workloads
from .problem import Problem


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def judge(net, cases, max_iter=300, tol=1e-8, opts=None):
    out = []
    for name, geo, n, sol in cases:
        pb = Problem(geo, n, 3, device=0, **(opts or {}))
        b = pb.rhs(sol.f, sol.u)
        learned.use(pb, False)
        _, st0 = pb.solve(b, tol=tol, max_iter=max_iter)
        learned.install(pb, net)
        _, st1 = pb.solve(b, tol=tol, max_iter=max_iter)
        out.append(dict(case=name, n=n, dofs=int(pb.n_dofs),
                        plain_iterations=st0["iterations"], plain_converged=st0["converged"],
                        plain_rel=st0["rel_residual"], plain_s=st0["seconds"],
                        learned_iterations=st1["iterations"], learned_converged=st1["converged"],
                        learned_rel=st1["rel_residual"], learned_s=st1["seconds"]))
        log(f"[judge] {name} n={n}: plain {st0['iterations']} its (rel {st0['rel_residual']:.1e}), "
            f"learned {st1['iterations']} its (rel {st1['rel_residual']:.1e})")
        pb.close()
    return out


def held_out_cases(sphere_sizes, union_sizes):
    """The sphere of the 96^3 workload and the eight-ball union of the 128^3
    one (neither among the training geometries) at the given sizes."""
    sph = workloads.problem("sphere96_q3")
    uni = workloads.problem("balls128_q3")
    return ([("sphere r=0.8", sph.geometry, n, sph.solution) for n in sphere_sizes] +
            [("8-ball union", uni.geometry, n, uni.solution) for n in union_sizes])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--geometries", type=int, default=200)
    ap.add_argument("--n", type=int, default=32)
    ap.add_argument("--iterates", default="0,3,8", help="Richardson steps before each sampled smoothing step")
    ap.add_argument("--geometry", default="ellipsoid", choices=["ellipsoid", "union", "mixed"],
                    help="training geometries: spheres/ellipsoids, 8-ball unions, or both alternating")
    ap.add_argument("--plain-form", action="store_true",
                    help="centre rule and per-level penalties instead of the stabilised 3D Q3 form")
    ap.add_argument("--draws", type=int, default=4)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--judge-sphere", default="32,48,96")
    ap.add_argument("--judge-union", default="32,64,128")
    ap.add_argument("--time-budget", type=float, default=240.0)
    ap.add_argument("--train-uv", type=int, default=1, help="1: train w, U, V; 0: relaxation weight only")
    args = ap.parse_args()
    dev = torch.device("cuda", 0)
    t0 = time.time()

    opts = {} if args.plain_form else dict(workloads.STABILISED_Q3)

    def factory(geo, n, p):
        return Problem(geo, n, p, device=0, **opts)

    its = tuple(int(k) for k in args.iterates.split(","))
    geom = {"ellipsoid": workloads.training_geometry, "union": workloads.training_union,
            "mixed": lambda s: workloads.training_union(s) if s % 2 else workloads.training_geometry(s)}[args.geometry]
    data = learned.generate(factory, range(1, args.geometries + 1), args.n, 3, its, args.draws, device=dev,
                            log=lambda m: None, geometry=geom)
    t_data = time.time() - t0
    log(f"[train] {data[0].shape[0]} samples from {args.geometries} geometries in {t_data:.1f} s")
    net = learned.MLP(data[0].shape[1], data[1].shape[1], 64, device=dev, omega=0.8, train_uv=bool(args.train_uv))
    t1 = time.time()
    hist = learned.train(net, data, epochs=args.epochs, batch=args.batch, lr=args.lr, log=log,
                         time_budget=args.time_budget)
    torch.cuda.synchronize()
    t_train = time.time() - t1
    net.save(args.out)
    sz = lambda a: [int(v) for v in a.split(",") if v]  # noqa: E731
    res = judge(net, held_out_cases(sz(args.judge_sphere), sz(args.judge_union)), opts=opts)
    print(json.dumps(dict(samples=int(data[0].shape[0]), geometries=args.geometries, n_train=args.n,
                          data_s=t_data, train_s=t_train, epochs=len(hist), loss_first=hist[0], loss_last=hist[-1],
                          loss_history=hist, judge=res)), flush=True)


if __name__ == "__main__":
    main()
