"""FP64 cases that exercise every neighbour-index path of the kernels (run by
tests/test_gpu_checked_build.py in a child process, once with the production
library and once with the index-checked one selected by RMRT_LIBRARY).

Usage: python tests/checked_cases.py OUT.npz
Writes every case's results to OUT.npz and prints one line per case with the
number of neighbour indices the checked build found out of range (-1 in the
production build), then the index-check self-test line in the checked build."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

import numpy as np  # noqa: E402

from gpu_util import WALLS, circle_mask  # noqa: E402
from paper_2206_00366_amd import rmrt as R  # noqa: E402


def fields(N, d, seed):
    rng = np.random.default_rng(seed)
    return 1.0 + 1e-3 * rng.uniform(-1, 1, N), 0.02 * rng.uniform(-1, 1, (d, N))


def violations(dom):
    return dom.checked_violations() if R.checked_build() else -1


def main(out_path):
    out = {}
    lines = []

    def single(name, prm, steps, solid=None, with_fne=False, launch=None, extra=None):
        p = R.make_params(**prm, storage="f64")
        n = prm["n"]
        N = n[0] * n[1] * n[2]
        d = 2 if prm["lattice"] in ("Q9", "Q5") else 3
        rho, u = fields(N, d, sum(map(ord, name)) % 1000)
        dom = R.Domain(p, rho, u if prm.get("equation", "NSE") == "NSE" else None,
                       solid=None if solid is None else solid.astype(np.uint8), with_fne=with_fne)
        if launch is not None:
            dom.set_launch(*launch)
        dom.step(steps)
        out[name + "/f"] = dom.populations().cpu().numpy()
        r, uu = dom.moments()
        out[name + "/rho"] = r.cpu().numpy()
        out[name + "/red"] = np.array(dom.reduce())
        if extra:
            extra(dom, name)
        lines.append(f"{name} {violations(dom)}")
        dom.close()

    def grads(dom, name):
        out[name + "/grad"] = dom.local_gradients(R.GRAD_STRAIN).cpu().numpy()
        dom.residual()                      # the first call sets the reference state
        dom.step(1)
        out[name + "/res"] = np.array([dom.residual()])

    single("q19_periodic_aa_odd", dict(lattice="Q19", n=(13, 11, 9), dx=(1.0, 0.5, 2.0), nu=0.03, pattern="AA"), 7,
           extra=grads)
    single("q27_walls_force_ab", dict(lattice="Q27", n=(21, 13, 9), dx=(1.0, 2.0, 1.0), nu=0.05,
                                      force=(1e-5, 0.0, 0.0), wall_faces=WALLS["yz"], pattern="AB"), 6)
    single("q9_solid_aa", dict(lattice="Q9", n=(40, 21, 1), dx=(1.0, 0.5, 1.0), nu=0.05, wall_faces=WALLS["y"],
                               pattern="AA"), 5, solid=circle_mask((40, 21, 1), (12, 10), 4), extra=grads)
    single("q9_solid_ab", dict(lattice="Q9", n=(40, 21, 1), dx=(1.0, 0.5, 1.0), nu=0.05, pattern="AB"), 4,
           solid=circle_mask((40, 21, 1), (20, 10), 5))
    single("q19_fne_walls_solid", dict(lattice="Q19", n=(17, 12, 10), dx=(1.0, 1.0, 2.0), nu=0.04,
                                       wall_faces=WALLS["yz"], pattern="AA"), 3,
           solid=circle_mask((17, 12, 10), (8, 6), 2), with_fne=True)
    single("q7_c_zero", dict(lattice="Q7", equation="NCDE", n=(11, 9, 7), dx=(1.0, 1.0, 2.0), D0=0.02, D2=0.5,
                             adv=(0.03, 0.01, -0.02), rho0=0.0, source=1e-4, pattern="AA"), 5)
    single("q9_ncde_c_zero_walls", dict(lattice="Q9", equation="NCDE", n=(33, 17, 1), dx=(1.0, 0.5, 1.0), D0=0.01,
                                        D2=1.0, adv=(0.05, 0.02, 0.0), rho0=0.0, c_zero=True, wall_faces=WALLS["y"],
                                        pattern="AA"), 5)
    single("q19_persistent_xcd", dict(lattice="Q19", n=(32, 24, 20), dx=(1.0, 0.5, 2.0), nu=0.03, pattern="AA"), 5,
           launch=(2, R.LAUNCH_PERSISTENT | R.LAUNCH_XCD_ORDER | R.LAUNCH_BUFFER_OFFSETS))
    single("q27_chunks_walls", dict(lattice="Q27", n=(45, 37, 29), nu=0.04, force=(1e-5, 0.0, 0.0),
                                    wall_faces=WALLS["yz"], pattern="AA"), 7)
    single("q27_central", dict(lattice="Q27", n=(11, 9, 7), dx=(1.0, 0.5, 2.0), nu=0.05, central=True,
                               wall_faces=WALLS["z"], pattern="AA"), 5)
    single("q19_hermite_walls", dict(lattice="Q19", n=(14, 9, 8), dx=(1.0, 2.0, 1.0), nu=0.05, s_hi=1.3,
                                     force=(1e-5, 0.0, 2e-6), wall_faces=WALLS["yz"], hermite=True,
                                     pattern="AA"), 5)
    single("q9_bhll_solid", dict(lattice="Q9", n=(40, 21, 1), dx=(1.0, 0.5, 1.0), nu=0.05, s_hi=1.2,
                                 force=(2e-5, 0.0, 0.0), wall_faces=WALLS["y"], bhll=True, pattern="AB"), 5,
           solid=circle_mask((40, 21, 1), (12, 10), 4))

    # a batch: ragged tile counts, walls, force, XCD chunks, domain groups; initial
    # state set at an odd parity (swapped-layout initialisation)
    dims = [(45, 37, 29), (16, 12, 9), (33, 50, 41)]
    prms = [R.make_params(lattice="Q27", n=n, nu=0.04, force=(1e-5, 0.0, 0.0), wall_faces=WALLS["yz"],
                          storage="f64", pattern="AA") for n in dims]
    b = R.Batch(prms)
    b.set_group_bytes(1)
    b.step(1)
    for k, n in enumerate(dims):
        rho, u = fields(n[0] * n[1] * n[2], 3, 40 + k)
        b.domains[k].set_fields(rho, u)
    b.step(6)
    for k in range(len(dims)):
        out[f"batch/{k}"] = b.domains[k].populations().cpu().numpy()
    out["batch/res"] = np.array(b.residuals())
    lines.append(f"batch {sum(violations(d) for d in b.domains) if R.checked_build() else -1}")
    b.close()

    np.savez(out_path, **out)
    for ln in lines:
        print("case", ln, flush=True)

    if R.checked_build():
        # the checks themselves: with the bound lowered below the node count,
        # the nodes above it count as out of range (every access stays inside
        # the buffers: a flagged index is replaced by the node's own)
        p = R.make_params(lattice="Q19", n=(16, 16, 16), nu=0.03, storage="f64", pattern="AA")
        N = 16 ** 3
        rho, u = fields(N, 3, 7)
        dom = R.Domain(p, rho, u)
        dom.step(2)
        clean = dom.checked_violations()
        dom.checked_set_limit(N - 300)
        dom.step(2)
        print(f"selftest {clean} {dom.checked_violations()}", flush=True)
        dom.close()


if __name__ == "__main__":
    main(sys.argv[1])
