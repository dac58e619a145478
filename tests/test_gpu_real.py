"""GPU parity of the real-orbital (Gamma-point) path.

Real orbitals (c(-G) = conj c(G)) give real pair densities; the library
packs two conduction orbitals per complex pair transform, unpacks real pair
rows in the cos/sin basis of the chi0 set and contracts in real FP64.  Every
output is compared with the FP64 oracle in the plane-wave basis (which the
library reports): orbitals, pair matrix elements, chi0 element by element
(1e-12 / 1e-10), eigenvalues, the projector C_s C_s^H, F_j and E_c (1e-10
relative), for an even and an odd number of conduction bands (the odd one
leaves the last packed orbital half empty), a ragged N_G, the medium
workload's geometry, and with the method's variants (basis from chi0's
eigenvectors, slab truncation, eps^-1).  The same system through the
general complex path gives the same E_c.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2405_20258_amd import ssrpa
    ctx = ssrpa.Context(0)
    yield torch, ssrpa, ctx
    ctx.close()


def tiny_real():
    from synth import systems as sy
    return sy.make_system(sy.TINY, 1000, real_orbitals=True)


def ragged_real():
    from synth import systems as sy
    # 18^3 grid, N_G = 80, 5 x 37 pairs (odd number of conduction bands)
    spec = sy.small_spec(a=9.0, fft=18, n_v=5, n_c=37, nsq_chi=6, e_psi=4.0)
    return sy.make_system(spec, 44, real_orbitals=True)


def _perm(g, s):
    from oracle import rpa
    idx = {tuple(int(x) for x in m): i for i, m in enumerate(g.gvectors())}
    mo = rpa.chi_gvectors(s.a, s.ecut_chi)
    return mo, np.array([idx[tuple(int(x) for x in m)] for m in mo])


@pytest.mark.parametrize("which", ["tiny", "ragged"])
def test_real_orbitals_and_pair_matrix(env, which):
    torch, ssrpa, ctx = env
    from oracle import rpa
    s = tiny_real() if which == "tiny" else ragged_real()
    g = ssrpa.System.from_synthetic(ctx, s)
    assert g.n_c == s.n_c
    mo, perm = _perm(g, s)
    n1, n2, n3 = s.fft
    psi = torch.empty((s.n_v + s.n_c, n3, n2, n1), dtype=torch.complex128,
                      device="cuda")
    g.orbitals_realspace(psi)
    torch.cuda.synchronize()
    ref_psi = rpa.orbitals_realspace(s.a, s.fft, s.miller, s.coeff)
    got = psi.cpu().numpy().transpose(0, 3, 2, 1)
    err = np.max(np.abs(got - ref_psi)) / np.max(np.abs(ref_psi))
    _log(f"real {which}: orbitals rel err {err:.2e}")
    assert err < 1e-13
    m_ref = rpa.pair_matrix_fft(s.a, s.fft, ref_psi[: s.n_v], ref_psi[s.n_v:], mo)
    for scaled in (False, True):
        ref = m_ref.reshape(s.n_v * s.n_c, -1)
        if scaled:
            ref = rpa.scaled_pair_matrix(s.a, m_ref, mo)
        out = torch.empty((s.n_v * s.n_c, len(mo)), dtype=torch.complex128,
                          device="cuda")
        g.pair_matrix(0, s.n_v, out, scaled=scaled)
        torch.cuda.synchronize()
        m = out.cpu().numpy()[:, perm]
        err = np.max(np.abs(m - ref)) / np.max(np.abs(ref))
        _log(f"real {which}: pair matrix scaled={scaled} rel err {err:.2e}")
        assert err < 1e-12
    g.close()


@pytest.mark.parametrize("which", ["tiny", "ragged"])
@pytest.mark.parametrize("symmetrized", [True, False])
def test_real_chi0_every_element(env, which, symmetrized):
    torch, ssrpa, ctx = env
    from oracle import rpa
    s = tiny_real() if which == "tiny" else ragged_real()
    g = ssrpa.System.from_synthetic(ctx, s)
    mo, perm = _perm(g, s)
    psi = rpa.orbitals_realspace(s.a, s.fft, s.miller, s.coeff)
    m = rpa.pair_matrix_fft(s.a, s.fft, psi[: s.n_v], psi[s.n_v:], mo)
    d = rpa.energy_factor(s.energy[: s.n_v], s.energy[s.n_v:], 0.0)
    ref = rpa.chi0(s.a, m, d)
    if symmetrized:
        ref = rpa.symmetrize_chi0(s.a, ref, mo)
    ng = len(mo)
    out = torch.empty((ng, ng), dtype=torch.complex128, device="cuda")
    g.chi0_static("fp64", out_dev=out, symmetrized=symmetrized)
    torch.cuda.synchronize()
    got = out.cpu().numpy()[np.ix_(perm, perm)]
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    _log(f"real {which} chi0 symmetrized={symmetrized}: rel err {err:.2e}")
    assert err < 1e-10
    assert np.max(np.abs(got - got.conj().T)) <= 1e-15 * np.max(np.abs(got))
    g.close()


@pytest.mark.parametrize("which,n_eig", [("tiny", 75), ("tiny", 304),
                                         ("ragged", 12), ("ragged", 80)])
def test_real_energy(env, which, n_eig):
    torch, ssrpa, ctx = env
    from oracle import rpa
    from synth import systems as sy
    s = tiny_real() if which == "tiny" else ragged_real()
    om, wt = sy.frequency_grid(16)
    g = ssrpa.System.from_synthetic(ctx, s)
    g.chi0_static("fp64")
    ng = g.n_g
    ref = rpa.correlation_energy(s.a, s.fft, s.miller, s.coeff, s.energy,
                                 s.n_v, s.ecut_chi, n_eig, om, wt)
    if n_eig < ng:
        mo, perm = _perm(g, s)
        basis = torch.empty((ng, n_eig), dtype=torch.complex128, device="cuda")
        lam = g.subspace(n_eig, basis)
        torch.cuda.synchronize()
        assert ref["gap"] > 1e-8
        assert np.max(np.abs(lam - ref["eigval"][:n_eig])) < \
            1e-10 * abs(ref["eigval"][0])
        c = basis.cpu().numpy()[perm]
        assert np.max(np.abs(c.conj().T @ c - np.eye(n_eig))) < 1e-12
        lr, vr = np.linalg.eigh(ref["chibar0"])
        pr = vr[:, :n_eig] @ vr[:, :n_eig].conj().T
        perr = np.max(np.abs(c @ c.conj().T - pr))
        _log(f"real {which} n_eig={n_eig}: projector err {perr:.2e}")
        assert perr < 1e-8
    ec, f = g.correlation_energy(n_eig, om, wt, "fp64")
    _log(f"real {which} n_eig={n_eig}: E_c gpu {ec!r} oracle {ref['ec']!r}")
    assert abs(ec - ref["ec"]) < 1e-10 * abs(ref["ec"])
    assert np.max(np.abs(f - ref["integrand"])) < \
        1e-10 * np.max(np.abs(ref["integrand"]))
    # the general complex path on the same orbitals
    gc = ssrpa.System.from_synthetic(ctx, s, real=False)
    gc.chi0_static("fp64")
    if n_eig < ng:
        gc.subspace(n_eig)
    ecc, _ = gc.correlation_energy(n_eig, om, wt, "fp64")
    assert abs(ecc - ec) < 1e-12 * abs(ec)
    gc.close()
    g.close()


def test_real_medium_geometry_chi0_every_element(env):
    """48^3, N_G = 3958 (31 x 31 tiles of 128), 2 x 256 pairs."""
    torch, ssrpa, ctx = env
    from oracle import rpa
    from synth import systems as sy
    s = sy.make_system(sy.MEDIUM, 2998, n_v=2, n_c=256, real_orbitals=True)
    g = ssrpa.System.from_synthetic(ctx, s)
    mo, perm = _perm(g, s)
    psi = rpa.orbitals_realspace(s.a, s.fft, s.miller, s.coeff)
    m = rpa.pair_matrix_fft(s.a, s.fft, psi[: s.n_v], psi[s.n_v:], mo)
    del psi
    w = rpa.scaled_pair_matrix(s.a, m, mo)
    d = rpa.pair_weights(s.energy, s.n_v, 0.0)
    ng = len(mo)
    out = torch.empty((ng, ng), dtype=torch.complex128, device="cuda")
    g.chi0_static("fp64", out_dev=out, symmetrized=True)
    torch.cuda.synchronize()
    dw = d[:, None] * w
    pt = torch.from_numpy(perm).cuda()
    err, big = 0.0, 0.0
    for r0 in range(0, ng, 1024):
        r1 = min(ng, r0 + 1024)
        ref = np.conj(w[:, r0:r1]).T @ dw / rpa.cell_volume(s.a)
        got = out[pt[r0:r1]][:, pt].cpu().numpy()
        err = max(err, float(np.max(np.abs(got - ref))))
        big = max(big, float(np.max(np.abs(ref))))
    _log(f"real medium geometry chi0: max err {err:.2e} of {big:.2e}")
    assert err < 1e-10 * big
    g.close()


@pytest.mark.parametrize("variant", ["chi0_basis", "slab", "eps_inv"])
def test_real_variants(env, variant):
    torch, ssrpa, ctx = env
    from oracle import rpa
    from synth import systems as sy
    s = tiny_real()
    om, wt = sy.frequency_grid(16)
    n_eig = 75
    if variant == "chi0_basis":
        g = ssrpa.System.from_synthetic(ctx, s)
        g.chi0_static("fp64")
        g.subspace(n_eig, kind="chi0")
        ec, _ = g.correlation_energy(n_eig, om, wt, "fp64")
        ref = rpa.correlation_energy_chi0_basis(
            s.a, s.fft, s.miller, s.coeff, s.energy, s.n_v, s.ecut_chi, n_eig,
            om, wt)
    elif variant == "slab":
        g = ssrpa.System.from_synthetic(ctx, s, truncation="slab")
        g.chi0_static("fp64")
        g.subspace(n_eig)
        ec, _ = g.correlation_energy(n_eig, om, wt, "fp64")
        ref = rpa.correlation_energy(s.a, s.fft, s.miller, s.coeff, s.energy,
                                     s.n_v, s.ecut_chi, n_eig, om, wt,
                                     truncation="slab")
    else:
        g = ssrpa.System.from_synthetic(ctx, s)
        g.chi0_static("fp64")
        g.subspace(n_eig)
        out = torch.empty((2, n_eig, n_eig), dtype=torch.complex128,
                          device="cuda")
        g.epsilon_inverse(n_eig, om[[0, 9]], out)
        torch.cuda.synchronize()
        ref = rpa.correlation_energy(s.a, s.fft, s.miller, s.coeff, s.energy,
                                     s.n_v, s.ecut_chi, n_eig, om[[0, 9]],
                                     wt[[0, 9]])
        for j in range(2):
            ev = np.sort(np.linalg.eigvalsh(out[j].cpu().numpy()))
            ev_ref = np.sort(np.linalg.eigvalsh(rpa.epsilon_inverse(
                ref["chis"][j])))
            err = np.max(np.abs(ev - ev_ref)) / np.max(np.abs(ev_ref))
            _log(f"real eps^-1 spectrum rel err {err:.2e}")
            assert err < 1e-10
        g.close()
        return
    _log(f"real {variant}: E_c gpu {ec!r} oracle {ref['ec']!r}")
    assert abs(ec - ref["ec"]) < 1e-10 * abs(ref["ec"])
    g.close()


def test_real_flag_is_checked(env):
    """Complex orbitals flagged real, and reduced precision on a real
    system, are refused."""
    torch, ssrpa, ctx = env
    from synth import systems as sy
    s = sy.make_system(sy.TINY, 1000)      # complex orbitals
    with pytest.raises(ssrpa.SsrpaError) as e:
        ssrpa.System.from_synthetic(ctx, s, real=True)
    assert e.value.status == ssrpa.ERR_ARG
    g = ssrpa.System.from_synthetic(ctx, tiny_real())
    with pytest.raises(ssrpa.SsrpaError) as e:
        g.chi0_static("fp32")
    assert e.value.status == ssrpa.ERR_ARG
    g.close()
