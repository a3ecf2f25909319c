"""Shared helpers of the GPU parity tests (HIP library vs FP64 oracle)."""
import sys

import numpy as np

import oracle as O
import paper_1009_0881_amd as P

# Parity bar over the first 50 iterations: |rel_err_gpu - rel_err_oracle| <= 1e-5
# and ||X_gpu - X_oracle||_F / ||X_oracle||_F <= 1e-4 for both factors.
TOL_REL_ERR = 1e-5
TOL_FACTOR = 1e-4


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def frob_rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def gpu_solve(M, V0, W0, h, w, r, levels, algo, cycle, xfer, T, tol=0.0, max_fine=0, **kw):
    m, n = M.shape
    pl = P.Plan(m=m, n=n, h=h, w=w, r=r, levels=levels, algo=algo, cycle=cycle, xfer=xfer,
                tol=tol, max_fine_iters=max_fine, **kw)
    Md, Vd, Wd = P.to_device(M, V0, W0)
    res = pl.solve(Md, Vd, Wd, T)
    rel, dep = pl.log(res["_workspace"])
    k = res["log_len"]
    V, Wn = P.factors_to_host(Vd, Wd)
    return res, rel[:k], dep[:k], V, Wn


def oracle_solve(M, V0, W0, h, w, r, levels, algo, cycle, xfer, T, tol=0.0, max_fine=0):
    res = O.solve(M, h, w, r, levels, P.ALGOS[algo] if isinstance(algo, str) else algo,
                  P.CYCLES[cycle] if isinstance(cycle, str) else cycle,
                  P.XFERS[xfer] if isinstance(xfer, str) else xfer, T, V0, W0,
                  tol=tol, max_fine_iters=max_fine)
    rel = np.array([e for _, e in res.log])
    dep = np.array([d for d, _ in res.log], dtype=np.int32)
    return res, rel, dep
