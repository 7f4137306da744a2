"""Write paper2d_oracle.json: the oracle's results for the paper's 2D case
(workloads.paper_2d: Table 1 and App. A, one-step scheme at Courant 0.9) on
grids from 600 x 300 to 6000 x 3000 bins (the paper's finest, 0.2 um bins,
for which it reports 1339 time steps).  Calls only the oracle; takes about
15 minutes on one core for the largest grid.

Usage: python tests/golden/make_paper2d.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from concurrent.futures import ThreadPoolExecutor  # noqa: E402

from oracle import ref  # noqa: E402
from paper_2411_00742_amd import workloads as W  # noqa: E402

SIZES = [(600, 300), (1200, 600), (2400, 1200), (3000, 1500), (6000, 3000)]


def one(nn):
    n1, n2 = nn
    p = W.paper_2d(n1, n2)
    t0 = time.time()
    r = ref.solve2d(p, 0, log_steps=0)
    return dict(n1=n1, n2=n2, steps=r["steps"], status=r["status"], t_final=r["t_final"],
                mom=r["mom"].tolist(), C=r["C"].tolist(), seconds=time.time() - t0)


def main():
    ref.lib()
    with ThreadPoolExecutor(max_workers=len(SIZES)) as ex:
        res = list(ex.map(one, SIZES))
    out = dict(source="oracle/pbe_oracle.cpp via oracle/ref.py solve2d, workloads.paper_2d(n1, n2) defaults",
               paper_steps_6000x3000=1339, cases=res)
    with open(os.path.join(HERE, "paper2d_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
    for r in res:
        print(r["n1"], r["n2"], r["steps"], f"{r['seconds']:.0f} s")


if __name__ == "__main__":
    main()
