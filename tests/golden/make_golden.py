"""Write oracle reference values for the tiny and medium workloads.

Calls only the FP64 oracle (oracle/rpa.py) on the seeded synthetic inputs
(synth/systems.py); nothing here touches the HIP library.  The paper prints
no worked numerical example (its performance data sit in figures and its
only table of energies is for Pt slabs whose wavefunctions are not
available), so these stored values are oracle outputs, not paper values.

Usage:  python tests/golden/make_golden.py tiny|medium [--no-full]
"""
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import rpa  # noqa: E402
from synth import systems as sy  # noqa: E402


def sample_pairs(rng, n_v, n_c, count):
    return [(int(rng.integers(n_v)), int(rng.integers(n_c)))
            for _ in range(count)]


def run(spec, seed, n_eigs, with_full, out_path):
    t0 = time.time()
    s = sy.make_system(spec, seed)
    om, wt = sy.frequency_grid(spec.n_freq)
    mchi = rpa.chi_gvectors(s.a, s.ecut_chi)
    ng = mchi.shape[0]
    psi = rpa.orbitals_realspace(s.a, s.fft, s.miller, s.coeff)
    nc = s.n_c
    w = np.empty((s.n_v * nc, ng), dtype=np.complex128)
    for v in range(s.n_v):
        m = rpa.pair_matrix_fft(s.a, s.fft, psi[v:v + 1], psi[s.n_v:], mchi)
        w[v * nc:(v + 1) * nc] = rpa.scaled_pair_matrix(s.a, m, mchi)
    del psi
    print(f"W {w.shape} {time.time() - t0:.1f}s", flush=True)

    def chibar_chunked(omega, ws):
        d = rpa.pair_weights(s.energy, s.n_v, omega)
        acc = np.zeros((ws.shape[1], ws.shape[1]), dtype=np.complex128)
        step = 32768
        for p0 in range(0, ws.shape[0], step):
            acc += rpa.chibar(s.a, ws[p0:p0 + step], d[p0:p0 + step])
        return acc

    cb0 = chibar_chunked(0.0, w)
    print(f"chibar0 {time.time() - t0:.1f}s", flush=True)
    rng = np.random.default_rng(12345)
    gi = rng.integers(ng, size=64)
    gj = rng.integers(ng, size=64)
    samples_chi = [[*map(int, mchi[i]), *map(int, mchi[j]),
                    float(cb0[i, j].real), float(cb0[i, j].imag)]
                   for i, j in zip(gi, gj)]
    samples_chi += [[*map(int, mchi[i]), *map(int, mchi[i]),
                     float(cb0[i, i].real), float(cb0[i, i].imag)]
                    for i in gi[:16]]
    pairs = sample_pairs(rng, s.n_v, s.n_c, 64)
    samples_w = []
    for (v, c) in pairs:
        for g in rng.integers(ng, size=4):
            val = w[v * nc + c, g]
            samples_w.append([v, c, *map(int, mchi[g]), float(val.real),
                              float(val.imag)])
    out = dict(
        workload=spec.name, seed=seed, n_freq=spec.n_freq, omega0=1.0,
        a=s.a, fft=list(s.fft), n_v=s.n_v, n_c=s.n_c, ecut_chi=s.ecut_chi,
        n_g=int(ng),
        chibar0_maxabs=float(np.max(np.abs(cb0))),
        chibar0_samples=samples_chi, w_samples=samples_w,
        provenance="FP64 oracle (oracle/rpa.py), written by "
                   "tests/golden/make_golden.py; symmetrized static "
                   "polarizability v^1/2 chi0 v^1/2 of Eq. (6), W = M v^1/2 "
                   "with M of Eq. (3); E_c of Eq. (1) in the static subspace "
                   "(Eqs. 7-8)",
        results={})
    lam_all = np.linalg.eigvalsh(cb0)
    out["eigval_all_head"] = [float(x) for x in lam_all[:max(n_eigs)]]
    for n_eig in n_eigs:
        lam, cs, gap = rpa.subspace(cb0, n_eig)
        ws = rpa.project(w, cs)
        f = np.array([rpa.trace_log_cholesky(chibar_chunked(float(o), ws))
                      for o in om])
        ec = rpa.quadrature(wt, f)
        out["results"][f"n_eig_{n_eig}"] = dict(
            n_eig=n_eig, ec=ec, integrand=[float(x) for x in f],
            eigval=[float(x) for x in lam], gap=float(gap))
        print(f"n_eig={n_eig} ec={ec!r} gap={gap:.3e} "
              f"{time.time() - t0:.1f}s", flush=True)
        with open(out_path, "w") as fh:
            json.dump(out, fh, indent=1)
    if with_full:
        f = np.empty(len(om))
        for j, o in enumerate(om):
            f[j] = rpa.trace_log_cholesky(chibar_chunked(float(o), w))
            print(f"full omega {j} {time.time() - t0:.1f}s", flush=True)
        ec = rpa.quadrature(wt, f)
        out["results"]["full"] = dict(n_eig=int(ng), ec=ec,
                                      integrand=[float(x) for x in f])
        print(f"full ec={ec!r}", flush=True)
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    which = sys.argv[1]
    full = "--no-full" not in sys.argv
    if which == "tiny":
        run(sy.TINY, sy.CONFIG_SEED_BASE[sy.TINY.name], [75, 150], full,
            os.path.join(HERE, "tiny.json"))
    elif which == "medium":
        run(sy.MEDIUM, sy.CONFIG_SEED_BASE[sy.MEDIUM.name], [400, 198, 792],
            full, os.path.join(HERE, "medium.json"))
    else:
        raise SystemExit("usage: make_golden.py tiny|medium [--no-full]")
