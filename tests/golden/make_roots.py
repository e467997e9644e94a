"""Writes the oracle roots that the full-size 11-level GPU tests compare
against.  Calls only the oracle and the input generators:

    python tests/golden/make_roots.py [name ...]

Each root is a JFNK solve of Algorithm 2 by the CPU oracle, in FP64, from LTE
populations, to a maximum scaled residual of 1e-12 (Sect. 2.2.2 stopping
rule); the file holds the populations [nz][nlev] as text with the problem,
the options and the oracle's final residual in its header.  Run with
OMP_NUM_THREADS=2 (the thread count of the stored files)."""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import nlte_oracle as O  # noqa: E402
from paper_2406_17234_amd import synth as S  # noqa: E402

# name -> (problem maker, solve options)
ROOTS = {
    "stream3_root": (lambda: S.stream_request(3),
                     dict(ftol=1e-12, rtol=1e-3, maxiter=80, max_krylov=300)),
    # the stress column: from LTE the GMRES path stalls (line searches down to
    # 1/256 from the 13th iteration), the BiCGSTAB path converges
    "chromo11_root": (S.chromo11,
                      dict(ftol=1e-12, rtol=1e-3, maxiter=60, max_krylov=100, krylov="bicgstab")),
    "chromo6_vel_root": (S.chromo6_vel,
                         dict(ftol=1e-12, rtol=1e-3, maxiter=80, max_krylov=300)),
}


def write(name):
    make, opts = ROOTS[name]
    p = make()
    tb = O.setup(p)
    t0 = time.time()
    s = O.solve(tb, **opts)
    dt = time.time() - t0
    if not s.converged:
        raise SystemExit(f"{name}: the oracle did not converge ({s.status}, {s.iters} iterations)")
    rho = float(np.max(np.abs(O.residual(tb, s.n).rho)))
    head = (f"oracle root of {p.name} dims={p.dims}\n"
            f"JFNK (Algorithm 2), FP64, LTE start, options {opts}\n"
            f"newton_iters={s.iters} f_calls={s.calls} max_scaled_residual={rho:.3e} "
            f"cpu_seconds={dt:.0f}\n"
            f"populations n[k][level], cm^-3")
    np.savetxt(os.path.join(HERE, name + ".txt"), s.n, fmt="%.17e", header=head)
    print(name, s.iters, s.calls, f"{rho:.2e}", f"{dt:.0f}s", flush=True)


def load(name):
    """The stored root [nz][nlev]."""
    return np.loadtxt(os.path.join(HERE, name + ".txt"))


if __name__ == "__main__":
    for n in sys.argv[1:] or sorted(ROOTS):
        write(n)
