"""Seeded synthetic inputs for the static-subspace RPA hot path.

This module builds the *inputs* of the problem only: a cubic cell, a
wavefunction plane-wave sphere, random orthonormal orbital coefficients, band
energies and an imaginary-frequency quadrature grid.  It holds none of the
method's arithmetic (no pair densities, no polarizability, no energies), so
that both the oracle and the HIP library can consume the same inputs without
sharing any code path of the method itself.

Recipe (the paper's own Pt-slab wavefunctions are not available, so these
synthetic systems stand in for them):

* Cell: simple cubic, lattice constant ``a`` bohr, volume a^3.
* Wavefunction sphere: Miller indices n with (2 pi / a)^2 |n|^2 / 2 <= E_psi
  (Hartree), ordered lexicographically.
* Coefficients: c_n(G) = (xi_1 + i xi_2) exp(-|G|^2 / (2 sigma^2)) with
  xi ~ N(0, 1), then a reduced QR so the bands are orthonormal.  Bands
  0..n_v-1 are valence (occupied), the rest conduction (empty).
* Energies (Hartree): valence sorted U[-1, 0]; conduction sorted
  0.1 + 4.9 u^(2/3), u ~ U[0, 1) (a free-electron sqrt(E) density of states
  from a 0.1 Ha band edge up to 5 Ha).
* Random numbers: numpy PCG64 ``default_rng(seed)`` drawn in the order
  Re xi, Im xi, eps_v, eps_c (real orbitals: xi, eps_v, eps_c).
* Real (time-reversal symmetric) orbitals: real coefficients in the cos/sin
  basis of each {G, -G} pair, a real QR, then c(-G) = conj c(G).
* Partial occupations: Fermi-Dirac factors at temperature kT around a
  chemical potential mu, values within 1e-12 of 0 or 1 set to 0 or 1.
* Chi0 cutoff: the midpoint between the closed shell |n|^2 <= nsq_chi and the
  next integer shell, so the G count is unambiguous.
* Frequencies: Gauss-Legendre nodes x_k, weights w_k on [-1, 1] (numpy's
  ``leggauss``) mapped to [0, inf) by omega = omega0 (1 + x) / (1 - x) with
  weight 2 omega0 w / (1 - x)^2, omega0 = 1 Ha.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np


@dataclasses.dataclass(frozen=True)
class SystemSpec:
    """Shape of one synthetic system."""

    name: str
    a: float            # cubic lattice constant, bohr
    fft: int            # wavefunction FFT grid per dimension
    n_v: int            # valence (occupied) bands
    n_c: int            # conduction (empty) bands
    nsq_chi: int        # chi0 basis: 0 < |n|^2 <= nsq_chi
    e_psi: float = 10.0  # wavefunction cutoff, Hartree
    sigma: float = 2.0   # Gaussian |G| decay of the random coefficients, 1/bohr
    n_freq: int = 16
    n_eig: int = 0       # default subspace size (0: full basis)
    valence_block: int = 0  # valence bands per block (0: all in one block)

    @property
    def n_bands(self) -> int:
        return self.n_v + self.n_c


# The workloads.  Sizes are stated explicitly; G counts follow from nsq_chi.
TINY = SystemSpec("tiny_fp64_a10_fft24_nv16_nc240_ng304", a=10.0, fft=24,
                  n_v=16, n_c=240, nsq_chi=17, n_freq=16, n_eig=75)
MEDIUM = SystemSpec("medium_fp64_a20_fft48_nv128_nc2048_ng3958", a=20.0,
                    fft=48, n_v=128, n_c=2048, nsq_chi=97, n_freq=16,
                    n_eig=400)
LARGE_SHARE = SystemSpec("large_share_a30_fft72_nv512_nc8192_ng15966",
                         a=30.0, fft=72, n_v=512, n_c=8192, nsq_chi=244,
                         n_freq=20, n_eig=1600, valence_block=32)

# k-mesh workload: the medium cell on the 2 x 2 x 2 mesh of kmesh_system,
# 32 x 512 bands per k-point (131072 pairs over the mesh), chi0 cutoff at
# 0.5 b^2 (97 + 0.4), evaluated at q = (1/2, 0, 0)
KMESH_MEDIUM = SystemSpec("kmesh_medium_a20_fft48_k8_nv32_nc512_q0.5",
                          a=20.0, fft=48, n_v=32, n_c=512, nsq_chi=97,
                          n_freq=16, n_eig=400)
KMESH_Q = (0.5, 0.0, 0.0)

CONFIG_SEED_BASE = {TINY.name: 1000, MEDIUM.name: 2000,
                    LARGE_SHARE.name: 3000, KMESH_MEDIUM.name: 4000}


def ecut_from_shell(a: float, nsq: int) -> float:
    """Cutoff (Ha) halfway between integer shells nsq and nsq + 1."""
    b = 2.0 * math.pi / a
    return 0.5 * b * b * (nsq + 0.5)


def sphere_miller(a: float, ecut: float) -> np.ndarray:
    """Miller indices n (int32, lexicographic) with (2pi/a)^2|n|^2/2 <= ecut."""
    b = 2.0 * math.pi / a
    nmax = int(math.floor(math.sqrt(2.0 * ecut) / b)) + 1
    r = np.arange(-nmax, nmax + 1)
    n1, n2, n3 = np.meshgrid(r, r, r, indexing="ij")
    nsq = n1 * n1 + n2 * n2 + n3 * n3
    keep = 0.5 * b * b * nsq <= ecut
    m = np.stack([n1[keep], n2[keep], n3[keep]], axis=1).astype(np.int32)
    return m


@dataclasses.dataclass
class System:
    """One concrete synthetic system (host arrays)."""

    spec: SystemSpec
    seed: int
    a: float
    fft: tuple
    miller: np.ndarray      # (n_pw, 3) int32
    coeff: np.ndarray       # (n_bands, n_pw) complex128, rows orthonormal
    energy: np.ndarray      # (n_bands,) float64, Hartree
    n_v: int
    n_c: int
    ecut_chi: float
    # occupation factors f_n in [0, 1] (None: insulator, f = 1 for the first
    # n_v bands and 0 for the rest); with occupations, n_v counts the bands
    # with f > 0
    occ: Optional[np.ndarray] = None
    real_orbitals: bool = False

    @property
    def n_pw(self) -> int:
        return int(self.miller.shape[0])

    @property
    def n_bands(self) -> int:
        return self.n_v + self.n_c


def _real_to_pw(miller: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Map real coefficients in the cos/sin basis to plane-wave coefficients.

    For each pair {G, -G} (G the lexicographically larger member) the real
    pair (x_G, x_-G) becomes c(G) = (x_G + i x_-G)/sqrt 2, c(-G) = conj c(G);
    G = 0 keeps its real coefficient.  The map is unitary, so orthonormal
    real columns give orthonormal orbitals with c(-G) = conj c(G), i.e.
    real orbitals psi(r) (time-reversal symmetric, as at the Gamma point).
    """
    index = {tuple(int(v) for v in m): i for i, m in enumerate(miller)}
    out = np.zeros(x.shape, dtype=np.complex128)
    r2 = 1.0 / math.sqrt(2.0)
    for i, m in enumerate(miller):
        t = tuple(int(v) for v in m)
        if t == (0, 0, 0):
            out[i] = x[i]
            continue
        j = index[(-t[0], -t[1], -t[2])]
        if t > (-t[0], -t[1], -t[2]):
            out[i] = (x[i] + 1j * x[j]) * r2
            out[j] = (x[i] - 1j * x[j]) * r2
    return out


def make_system(spec: SystemSpec, seed: int, n_v: Optional[int] = None,
                n_c: Optional[int] = None, qr: str = "numpy",
                real_orbitals: bool = False) -> System:
    """Draw one seeded synthetic system of the given shape.

    qr="torch" orthonormalizes on the GPU (torch.linalg.qr) for large inputs;
    the random numbers are the same, the orbitals agree with the numpy QR up
    to rounding and per-band phases.

    real_orbitals=True draws real coefficients xi ~ N(0, 1) (one draw per
    plane wave and band, no imaginary part) in the cos/sin basis, takes a
    real reduced QR and maps them to plane waves with c(-G) = conj c(G)
    (see _real_to_pw); the energies follow as before.
    """
    n_v = spec.n_v if n_v is None else n_v
    n_c = spec.n_c if n_c is None else n_c
    nb = n_v + n_c
    miller = sphere_miller(spec.a, spec.e_psi)
    n_pw = miller.shape[0]
    if nb > n_pw:
        raise ValueError(f"{nb} bands exceed the {n_pw} plane waves")
    b = 2.0 * math.pi / spec.a
    g2 = (b * b) * np.sum(miller.astype(np.float64) ** 2, axis=1)
    envelope = np.exp(-g2 / (2.0 * spec.sigma ** 2))
    rng = np.random.default_rng(seed)
    xr = rng.standard_normal((n_pw, nb))
    xi = None if real_orbitals else rng.standard_normal((n_pw, nb))
    eps_v = np.sort(rng.uniform(-1.0, 0.0, n_v))
    u = rng.uniform(0.0, 1.0, n_c)
    eps_c = np.sort(0.1 + 4.9 * u ** (2.0 / 3.0))
    if real_orbitals:
        q, _ = np.linalg.qr(xr * envelope[:, None], mode="reduced")
        coeff = np.ascontiguousarray(_real_to_pw(miller, q).T)
        energy = np.concatenate([eps_v, eps_c]).astype(np.float64)
        return System(spec=spec, seed=seed, a=spec.a, fft=(spec.fft,) * 3,
                      miller=miller, coeff=coeff, energy=energy, n_v=n_v,
                      n_c=n_c, ecut_chi=ecut_from_shell(spec.a, spec.nsq_chi),
                      real_orbitals=True)
    z = (xr + 1j * xi) * envelope[:, None]
    if qr == "torch":
        import torch
        q = torch.linalg.qr(torch.from_numpy(z).to("cuda"), mode="reduced")[0]
        coeff = np.ascontiguousarray(q.T.cpu().numpy())
        del q
    else:
        q, _ = np.linalg.qr(z, mode="reduced")
        coeff = np.ascontiguousarray(q.T)  # (nb, n_pw): one band per row
    energy = np.concatenate([eps_v, eps_c]).astype(np.float64)
    return System(spec=spec, seed=seed, a=spec.a, fft=(spec.fft,) * 3,
                  miller=miller, coeff=coeff, energy=energy, n_v=n_v,
                  n_c=n_c, ecut_chi=ecut_from_shell(spec.a, spec.nsq_chi))


def kmesh_system(a: float, fft: int, n_v: int, n_c: int, nsq_chi: int,
                 seed: int, e_psi: float = 4.0, sigma: float = 2.0):
    """A shifted 2 x 2 x 2 k mesh {+-1/4}^3 (fractions of the reciprocal
    vectors), weights 1/8, time-reversal symmetric: for each k of the half
    set (k_x = +1/4) random orbitals on the sphere |k + G|^2/2 <= e_psi
    (Gaussian |k + G| decay, reduced QR) and energies as in make_system; at
    -k the coefficients c_-k(G) = conj c_k(-G) and the same energies.
    Returns (kpoints: list of dicts miller, coeff, energy, n_v, weight,
    kfrac; ecut_chi), drawn per half-set k-point in order with
    default_rng(seed)."""
    b = 2.0 * math.pi / a
    rng = np.random.default_rng(seed)
    half = [(0.25, sy, sz) for sy in (0.25, -0.25) for sz in (0.25, -0.25)]
    kpts = {}
    for kf in half:
        kv = np.array(kf)
        nmax = int(math.floor(math.sqrt(2.0 * e_psi) / b)) + 2
        r = np.arange(-nmax, nmax + 1)
        n1, n2, n3 = np.meshgrid(r, r, r, indexing="ij")
        m = np.stack([n1.ravel(), n2.ravel(), n3.ravel()], axis=1)
        kg2 = b * b * np.sum((m + kv[None, :]) ** 2, axis=1)
        m = m[0.5 * kg2 <= e_psi].astype(np.int32)
        kg2 = b * b * np.sum((m + kv[None, :]) ** 2, axis=1)
        nb = n_v + n_c
        if nb > len(m):
            raise ValueError("too many bands for the sphere")
        z = (rng.standard_normal((len(m), nb)) + 1j *
             rng.standard_normal((len(m), nb))) * np.exp(
                 -kg2 / (2.0 * sigma ** 2))[:, None]
        q, _ = np.linalg.qr(z, mode="reduced")
        eps_v = np.sort(rng.uniform(-1.0, 0.0, n_v))
        eps_c = np.sort(0.1 + 4.9 * rng.uniform(0.0, 1.0, n_c) ** (2.0 / 3.0))
        e = np.concatenate([eps_v, eps_c])
        kpts[kf] = dict(miller=m, coeff=np.ascontiguousarray(q.T), energy=e,
                        n_v=n_v, weight=1.0 / 8.0, kfrac=np.array(kf))
        mk = kf
        km = tuple(-x for x in mk)
        # time reversal: c_-k(G) = conj c_k(-G), on the sphere -S(k)
        mneg = (-m).astype(np.int32)
        kpts[km] = dict(miller=mneg, coeff=np.ascontiguousarray(np.conj(q.T)),
                        energy=e.copy(), n_v=n_v, weight=1.0 / 8.0,
                        kfrac=np.array(km))
    order = sorted(kpts.keys())
    return [kpts[k] for k in order], ecut_from_shell(a, nsq_chi)


def kmesh_partners(kpoints, q0, seed: int, e_psi: float, a: float,
                   sigma: float = 2.0):
    """Weight-0 k-points at k + q0 for every k of `kpoints` (a small-q0
    evaluation of the q -> 0 term): random orbitals on the sphere
    |k + q0 + G|^2/2 <= e_psi and energies drawn as in kmesh_system, with
    default_rng(seed), in the order of `kpoints`."""
    b = 2.0 * math.pi / a
    rng = np.random.default_rng(seed)
    out = []
    for k in kpoints:
        kv = np.asarray(k["kfrac"], dtype=np.float64) + np.asarray(q0)
        nmax = int(math.floor(math.sqrt(2.0 * e_psi) / b)) + 2
        r = np.arange(-nmax, nmax + 1)
        n1, n2, n3 = np.meshgrid(r, r, r, indexing="ij")
        m = np.stack([n1.ravel(), n2.ravel(), n3.ravel()], axis=1)
        kg2 = b * b * np.sum((m + kv[None, :]) ** 2, axis=1)
        m = m[0.5 * kg2 <= e_psi].astype(np.int32)
        kg2 = b * b * np.sum((m + kv[None, :]) ** 2, axis=1)
        n_v = int(k["n_v"])
        nb = len(k["energy"])
        z = (rng.standard_normal((len(m), nb)) + 1j *
             rng.standard_normal((len(m), nb))) * np.exp(
                 -kg2 / (2.0 * sigma ** 2))[:, None]
        qr, _ = np.linalg.qr(z, mode="reduced")
        eps_v = np.sort(rng.uniform(-1.0, 0.0, n_v))
        eps_c = np.sort(0.1 + 4.9 * rng.uniform(0.0, 1.0, nb - n_v) ** (2.0 / 3.0))
        out.append(dict(miller=m, coeff=np.ascontiguousarray(qr.T),
                        energy=np.concatenate([eps_v, eps_c]), n_v=n_v,
                        weight=0.0, kfrac=kv))
    return out


def kmesh_q_map(kpoints, q):
    """For q (fractions) on the mesh: kq[i], g0[i] with k_i + q = k_kq[i] + g0[i]."""
    kq, g0 = [], []
    ks = [np.asarray(k["kfrac"]) for k in kpoints]
    for k in ks:
        t = k + np.asarray(q)
        for j, kk in enumerate(ks):
            d = t - kk
            if np.all(np.abs(d - np.round(d)) < 1e-12):
                kq.append(j)
                g0.append(np.round(d).astype(np.int32))
                break
        else:
            raise ValueError("q is not on the mesh")
    return np.array(kq, dtype=np.int32), np.array(g0, dtype=np.int32)


def fermi_dirac_occupations(energy: np.ndarray, mu: float, kt: float,
                            cut: float = 1e-12) -> np.ndarray:
    """Finite-temperature occupations f = 1 / (1 + exp((e - mu) / kT)).

    Values within `cut` of 1 or 0 are set to exactly 1 or 0, so that the
    fully occupied and the empty bands are well defined.  Energies must be
    ascending; f is then non-increasing.
    """
    x = (np.asarray(energy, dtype=np.float64) - mu) / kt
    f = 0.5 * (1.0 - np.tanh(0.5 * x))   # 1/(1 + e^x) without overflow
    f[f > 1.0 - cut] = 1.0
    f[f < cut] = 0.0
    return f


def with_occupations(s: System, occ: np.ndarray) -> System:
    """The same orbitals and energies with occupation factors `occ`.

    n_v becomes the number of bands with f > 0 and n_c the rest, so the
    bands keep their order; the library derives the partially occupied set
    from `occ` itself.
    """
    occ = np.asarray(occ, dtype=np.float64)
    n_val = int(np.count_nonzero(occ > 0.0))
    return dataclasses.replace(s, occ=occ, n_v=n_val, n_c=s.n_bands - n_val)


def small_spec(a: float = 8.0, fft: int = 16, n_v: int = 4, n_c: int = 28,
               nsq_chi: int = 5, e_psi: float = 4.0, n_freq: int = 16,
               name: str = "small") -> SystemSpec:
    """A very small system for brute-force checks."""
    return SystemSpec(name, a=a, fft=fft, n_v=n_v, n_c=n_c, nsq_chi=nsq_chi,
                      e_psi=e_psi, n_freq=n_freq)


def frequency_grid(n: int, omega0: float = 1.0):
    """Gauss-Legendre rule mapped to [0, inf): (omega, weight) float64."""
    x, w = np.polynomial.legendre.leggauss(n)
    omega = omega0 * (1.0 + x) / (1.0 - x)
    weight = 2.0 * omega0 * w / (1.0 - x) ** 2
    return omega.astype(np.float64), weight.astype(np.float64)


def alias_free_grid(miller_psi: np.ndarray, nsq_chi: int) -> int:
    """Smallest 2^i 3^j grid with N >= 2 max|n_psi| + max|n_chi| + 1."""
    npsi = int(np.max(np.abs(miller_psi)))
    nchi = int(math.floor(math.sqrt(nsq_chi)))
    need = 2 * npsi + nchi + 1
    best = None
    for i in range(0, 12):
        for j in range(0, 8):
            v = (2 ** i) * (3 ** j)
            if v >= need and (best is None or v < best):
                best = v
    return best


def serving_stream(n_requests: int = 64, rate: float = 4.0, seed: int = 5000,
                   nv_range=(16, 256), ng_range=(500, 6000),
                   eig_frac: float = 0.1, n_freq: int = 16):
    """Request descriptors for the mixed serving stream.

    Arrivals are Poisson (exponential gaps at ``rate`` per second).  Each
    request has N_v ~ U{nv_range}, N_c = 16 N_v, a chi0 size drawn uniformly
    from ``ng_range`` and rounded to the nearest closed shell, N_eig =
    round(eig_frac N_G), and FP64 or BF16x3 precision with probability 1/2.
    The cell is sized so that the wavefunction sphere holds about five plane
    waves per band.
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, n_requests)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(n_requests):
        n_v = int(rng.integers(nv_range[0], nv_range[1] + 1))
        n_c = 16 * n_v
        ng_target = float(rng.uniform(ng_range[0], ng_range[1]))
        prec = "fp64" if rng.uniform() < 0.5 else "bf16x3"
        nb = n_v + n_c
        # |n|^2 <= (a sqrt(2 E_psi) / 2 pi)^2 holds ~ (4 pi / 3) r^3 points
        a = (5.0 * nb / 1.5104) ** (1.0 / 3.0)
        nsq = _closest_shell(ng_target)
        out.append(dict(index=i, arrival=float(t[i]), n_v=n_v, n_c=n_c,
                        a=float(a), nsq_chi=nsq, precision=prec,
                        n_freq=n_freq, eig_frac=eig_frac,
                        seed=seed + 1 + i))
    return out


def _closest_shell(ng_target: float) -> int:
    best, best_err = 1, None
    counts = _shell_counts(120)
    for nsq in range(1, len(counts)):
        err = abs(counts[nsq] - ng_target)
        if best_err is None or err < best_err:
            best, best_err = nsq, err
    return best


_SHELLS = None


def _shell_counts(nmax: int):
    global _SHELLS
    if _SHELLS is None:
        r = np.arange(-nmax, nmax + 1)
        sq = r * r
        tot = (sq[:, None, None] + sq[None, :, None] + sq[None, None, :])
        lim = 400
        hist = np.bincount(tot[tot <= lim].ravel(), minlength=lim + 1)
        _SHELLS = np.cumsum(hist) - 1  # exclude G = 0
    return _SHELLS


def serving_system(req: dict, qr: str = "numpy") -> tuple:
    """Concrete (System, n_eig) for one serving request."""
    a = req["a"]
    spec = SystemSpec(f"serve_{req['index']}", a=a, fft=8, n_v=req["n_v"],
                      n_c=req["n_c"], nsq_chi=req["nsq_chi"],
                      n_freq=req["n_freq"])
    miller = sphere_miller(a, spec.e_psi)
    grid = alias_free_grid(miller, spec.nsq_chi)
    spec = dataclasses.replace(spec, fft=grid)
    sysm = make_system(spec, req["seed"], qr=qr)
    n_g = int(_shell_counts(120)[spec.nsq_chi])
    n_eig = max(1, int(round(req["eig_frac"] * n_g)))
    return sysm, n_eig
