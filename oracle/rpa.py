"""Plain FP64 CPU oracle for static-subspace RPA correlation energies.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library may import, call or
link this module; only the tests, the smoke check and the CPU-baseline leg of
the benchmark use it.  It shares no code with the HIP path.

Everything here follows the paper's Method section (Weinberg et al.,
"Static Subspace Approximation for Random Phase Approximation Correlation
Energies: Implementation and Performance", arXiv:2405.20258), restricted to
one q-point (q = 0), the Gamma point (one k-point, weight 1) and spin
degeneracy (the factor 2 of Eq. 2); occupations are those of an insulator
(f_v = 1, f_c = 0) or, with partial occupations, given per band (Eqs. 4-6):

* Eq. (1)  E_c = int_0^inf d omega / (2 pi) Tr[ln(1 - chi0 v) + chi0 v]
* Eq. (3)  plane-wave matrix elements M_vc(G) = <psi_v | e^{iG.r} | psi_c>
* Eq. (5)/(2) energy factor Delta_vc(i omega)
* Eq. (6)  chi0_GG' = (1/Omega) sum_vc conj(M_vc(G)) Delta_vc M_vc(G')
* Static subspace: the basis C_s holds the N_eig eigenvectors of the static
  response with the largest |eigenvalue|; Eq. (7) M_s = M C_s and
  Eq. (8) chi0_s = M_s^H Delta M_s.
* The trace of the logarithm is taken as the log of a determinant
  (Implementation section, last paragraph), here from a Cholesky factor,
  with an LU factor as a cross-check.

Readings taken where the paper is silent or ambiguous (each is listed in
the design notes):

* Delta.  Eq. (5) prints only the resonant term 2 g (f_c - f_v) /
  (e_c - e_v - i w); Eq. (2) sums n, n' over all bands, which adds the
  anti-resonant partner.  With g = 1, f_v = 1, f_c = 0 the sum of the two is
  Delta_vc(i w) = -4 de / (de^2 + w^2), de = e_c - e_v > 0, real and
  negative, so chi0(i w) is Hermitian negative semidefinite.
* 1/Omega appears once, inside chi0 (Eqs. 2, 6); v(G) = 4 pi / |G|^2.
* The subspace basis is built from v^1/2 chi0(0) v^1/2 (a similarity
  transform of chi0 v, so Tr ln(1 - chi0 v) = ln det(1 - v^1/2 chi0 v^1/2)).
* The G = 0 component is excluded from the chi0 basis.
* "Greatest absolute eigenvalues" of a negative semidefinite matrix are the
  most negative ones; eigenvalues are returned in ascending order.
* The frequency quadrature is an input (omega_j, w_j); the default is
  Gauss-Legendre mapped to [0, inf) by omega = omega0 (1 + x)/(1 - x).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft
import scipy.linalg

# ---------------------------------------------------------------------------
# Cell, G sets and the Coulomb kernel
# ---------------------------------------------------------------------------


def cell_volume(a: float) -> float:
    """Volume Omega of the simple cubic cell (the V of Eq. 2)."""
    return float(a) ** 3


def recip_unit(a: float) -> float:
    """Length of the reciprocal lattice vectors of a cubic cell, 2 pi / a."""
    return 2.0 * math.pi / float(a)


def chi_gvectors(a: float, ecut_chi: float) -> np.ndarray:
    """Miller indices of the chi0 basis: G != 0 with |G|^2/2 <= ecut_chi.

    The basis of the polarizability is the set of reciprocal lattice vectors
    (Method, after Eq. 1).  Order: lexicographic in (n1, n2, n3).
    """
    b = recip_unit(a)
    nmax = int(math.floor(math.sqrt(2.0 * ecut_chi) / b)) + 1
    out = []
    for n1 in range(-nmax, nmax + 1):
        for n2 in range(-nmax, nmax + 1):
            for n3 in range(-nmax, nmax + 1):
                nsq = n1 * n1 + n2 * n2 + n3 * n3
                if nsq == 0:
                    continue
                if 0.5 * b * b * nsq <= ecut_chi:
                    out.append((n1, n2, n3))
    return np.array(out, dtype=np.int64).reshape(-1, 3)


def gnorm2(a: float, miller: np.ndarray) -> np.ndarray:
    """|G|^2 for Miller indices of a cubic cell."""
    b = recip_unit(a)
    m = np.asarray(miller, dtype=np.float64)
    return b * b * np.sum(m * m, axis=1)


def coulomb(a: float, miller: np.ndarray) -> np.ndarray:
    """Bare Coulomb kernel v(G) = 4 pi / |G|^2 (G != 0), Hartree atomic units."""
    return 4.0 * math.pi / gnorm2(a, miller)


def coulomb_slab(a: float, miller: np.ndarray) -> np.ndarray:
    """Coulomb kernel truncated along z for a slab (Computational Details:
    truncation along the axis normal to the surface).

    The interaction is cut at |z| = z_c = a/2 (half the cell height), so a
    charge in the slab does not see its periodic images along z:
    v(G) = int d^2 rho int_{-z_c}^{z_c} dz e^{-iG.r} / |r|
         = 4 pi / |G|^2 [1 - e^{-G_par z_c} cos(G_z z_c)],
    G_par = (G_x^2 + G_y^2)^1/2 (the term in sin(G_z z_c) vanishes since
    G_z z_c = pi n).  At G_par = 0 the limit 4 pi / G_z^2 [1 - cos(G_z z_c)]
    holds, which is zero for even n.
    """
    b = recip_unit(a)
    m = np.asarray(miller, dtype=np.float64)
    gpar = b * np.sqrt(m[:, 0] ** 2 + m[:, 1] ** 2)
    gz = b * m[:, 2]
    zc = 0.5 * float(a)
    g2 = gpar * gpar + gz * gz
    return 4.0 * math.pi / g2 * (1.0 - np.exp(-gpar * zc) * np.cos(gz * zc))


def coulomb_kernel(a: float, miller: np.ndarray, truncation=None) -> np.ndarray:
    """v(G): bare (truncation None) or "slab" (truncated along z)."""
    if truncation is None:
        return coulomb(a, miller)
    if truncation == "slab":
        return coulomb_slab(a, miller)
    raise ValueError(f"unknown truncation {truncation!r}")


# ---------------------------------------------------------------------------
# Orbitals and plane-wave matrix elements (Eq. 3)
# ---------------------------------------------------------------------------


def orbitals_realspace(a, fft, miller_psi, coeff) -> np.ndarray:
    """psi_n(r_j) = Omega^-1/2 sum_G c_n(G) e^{i G.r_j} on the FFT grid.

    Grid points r_j = a (j1/N1, j2/N2, j3/N3); array layout [band, j1, j2, j3].
    Uses the library inverse FFT, whose kernel is e^{+2 pi i n.j/N} / N^3.
    """
    n1, n2, n3 = fft
    nb = coeff.shape[0]
    box = np.zeros((nb, n1, n2, n3), dtype=np.complex128)
    m = np.asarray(miller_psi)
    box[:, m[:, 0] % n1, m[:, 1] % n2, m[:, 2] % n3] = coeff
    psi = scipy.fft.ifftn(box, axes=(1, 2, 3), workers=-1)
    psi *= (n1 * n2 * n3) / math.sqrt(cell_volume(a))
    return psi


def pair_matrix_fft(a, fft, psi_v, psi_c, miller_chi) -> np.ndarray:
    """M_vc(G) of Eq. (3) at q = 0 from real-space pair densities.

    rho_vc(r_j) = conj(psi_v(r_j)) psi_c(r_j);
    M_vc(G) = (Omega / N) sum_j rho_vc(r_j) e^{+i G.r_j}, N = N1 N2 N3.
    The grid sum equals the cell integral when N_i >= 2 max|n_psi,i| +
    max|n_chi,i| + 1 (no aliasing).  Returns [v, c, G].
    """
    n1, n2, n3 = fft
    m = np.asarray(miller_chi)
    out = np.empty((psi_v.shape[0], psi_c.shape[0], m.shape[0]),
                   dtype=np.complex128)
    omega = cell_volume(a)
    for iv in range(psi_v.shape[0]):
        rho = np.conj(psi_v[iv])[None] * psi_c
        # sum_j rho e^{+2 pi i n.j/N} = N * ifftn(rho)[n]
        f = scipy.fft.ifftn(rho, axes=(1, 2, 3), workers=-1)
        out[iv] = omega * f[:, m[:, 0] % n1, m[:, 1] % n2, m[:, 2] % n3]
    return out


def pair_matrix_convolution(miller_psi, coeff_v, coeff_c, miller_chi):
    """M_vc(G) of Eq. (3) as a plane-wave convolution, no grid at all.

    <psi_v| e^{iG.r} |psi_c> = sum_{G1} conj(c_v(G1)) c_c(G1 - G) with both
    G1 and G1 - G in the wavefunction sphere.  Returns [v, c, G].
    """
    mp = np.asarray(miller_psi, dtype=np.int64)
    index = {tuple(x): i for i, x in enumerate(mp)}
    mc = np.asarray(miller_chi, dtype=np.int64)
    out = np.zeros((coeff_v.shape[0], coeff_c.shape[0], mc.shape[0]),
                   dtype=np.complex128)
    for ig, g in enumerate(mc):
        src, dst = [], []
        for i1, g1 in enumerate(mp):
            j = index.get((g1[0] - g[0], g1[1] - g[1], g1[2] - g[2]))
            if j is not None:
                src.append(i1)
                dst.append(j)
        if src:
            cv = np.conj(coeff_v[:, src])       # (nv, k)
            cc = coeff_c[:, dst]                 # (nc, k)
            out[:, :, ig] = cv @ cc.T
    return out


def pair_matrix_realspace_bruteforce(a, fft, miller_psi, coeff_v, coeff_c,
                                     miller_chi) -> np.ndarray:
    """M_vc(G) by explicit real-space sums, no FFT anywhere (tiny inputs).

    psi(r_j) is summed plane wave by plane wave, the pair density formed
    point by point and its Fourier component summed over the grid.
    """
    n1, n2, n3 = fft
    j = np.stack(np.meshgrid(np.arange(n1) / n1, np.arange(n2) / n2,
                             np.arange(n3) / n3, indexing="ij"), -1)
    j = j.reshape(-1, 3)                                   # fractional r
    mp = np.asarray(miller_psi, dtype=np.float64)
    phase_psi = np.exp(2j * math.pi * (j @ mp.T))          # (Nr, npw)
    omega = cell_volume(a)
    psi_v = (phase_psi @ coeff_v.T) / math.sqrt(omega)     # (Nr, nv)
    psi_c = (phase_psi @ coeff_c.T) / math.sqrt(omega)     # (Nr, nc)
    mc = np.asarray(miller_chi, dtype=np.float64)
    phase_g = np.exp(2j * math.pi * (j @ mc.T))            # (Nr, NG)
    nr = j.shape[0]
    out = np.empty((coeff_v.shape[0], coeff_c.shape[0], mc.shape[0]),
                   dtype=np.complex128)
    for iv in range(coeff_v.shape[0]):
        rho = np.conj(psi_v[:, iv])[:, None] * psi_c       # (Nr, nc)
        out[iv] = (omega / nr) * (rho.T @ phase_g)
    return out


# ---------------------------------------------------------------------------
# Energy factor and polarizability (Eqs. 2, 5, 6)
# ---------------------------------------------------------------------------


def energy_factor(eps_v, eps_c, omega: float) -> np.ndarray:
    """Delta_vc(i omega), [v, c], for f_v = 1, f_c = 0, g = 1, spin 2.

    Resonant plus anti-resonant terms of Eq. (2):
    -2/(de - i w) - 2/(de + i w) = -4 de / (de^2 + w^2), de = e_c - e_v.
    """
    de = np.asarray(eps_c)[None, :] - np.asarray(eps_v)[:, None]
    return -4.0 * de / (de * de + omega * omega)


def band_sets(occ):
    """Valence set V (f > 0) and conduction set C (f < 1), band indices.

    Eq. (4) sorts the non-zero terms of Eq. (2) into (occupied, empty),
    (occupied, partial), (partial, empty) and (partial, partial) pairs; the
    index change before Eq. (5) lets v run over occupied and partially
    occupied bands and c over partially occupied and empty ones.
    """
    f = np.asarray(occ, dtype=np.float64)
    return np.nonzero(f > 0.0)[0], np.nonzero(f < 1.0)[0]


def energy_factor_occ(eps, occ, omega: float) -> np.ndarray:
    """Delta_vc(i omega) over V x C, [v, c], with occupation factors.

    For two bands n < m (ascending energies) Eq. (2) holds the ordered terms
    (n, m) and (m, n): 2 (f_m - f_n) / (e_m - e_n - i w) and
    2 (f_n - f_m) / (e_n - e_m - i w), whose sum is
    -4 (f_n - f_m) de / (de^2 + w^2), de = e_m - e_n (the occupied-empty
    case f_n = 1, f_m = 0 gives energy_factor).  Each unordered pair is
    counted once: a pair of two partially occupied bands appears in V x C in
    both orders, and the order with v >= c (band index) gets 0.  A pair with
    equal occupations contributes 0; unequal occupations at equal energies
    have no static limit and are rejected.
    """
    f = np.asarray(occ, dtype=np.float64)
    e = np.asarray(eps, dtype=np.float64)
    v, c = band_sets(f)
    de = e[c][None, :] - e[v][:, None]
    df = f[v][:, None] - f[c][None, :]
    keep = (v[:, None] < c[None, :]) & (df != 0.0)
    if np.any(keep & (de <= 0.0)):
        raise ValueError("bands with different occupations need ascending, "
                         "distinct energies")
    out = np.zeros(de.shape)
    out[keep] = -4.0 * df[keep] * de[keep] / (de[keep] ** 2 + omega * omega)
    return out


def scaled_pair_matrix(a, m_vcg, miller_chi, truncation=None) -> np.ndarray:
    """W_p(G) = M_p(G) v(G)^1/2 as a (pairs, G) matrix, pair p = v N_c + c."""
    nv, nc, ng = m_vcg.shape
    return (m_vcg.reshape(nv * nc, ng)
            * np.sqrt(coulomb_kernel(a, miller_chi, truncation))[None, :])


def chi0(a, m_vcg, delta_vc) -> np.ndarray:
    """chi0_GG' = (1/Omega) sum_vc conj(M_vc(G)) Delta_vc M_vc(G')  (Eq. 6)."""
    nv, nc, ng = m_vcg.shape
    mm = m_vcg.reshape(nv * nc, ng)
    d = np.asarray(delta_vc).reshape(nv * nc)
    return (np.conj(mm).T * d[None, :]) @ mm / cell_volume(a)


def chibar(a, w, delta_p) -> np.ndarray:
    """v^1/2 chi0 v^1/2 = (1/Omega) W^H diag(Delta) W."""
    return (np.conj(w).T * np.asarray(delta_p)[None, :]) @ w / cell_volume(a)


def symmetrize_chi0(a, chi, miller_chi, truncation=None) -> np.ndarray:
    """v^1/2 chi0 v^1/2 from chi0."""
    s = np.sqrt(coulomb_kernel(a, miller_chi, truncation))
    return s[:, None] * chi * s[None, :]


# ---------------------------------------------------------------------------
# Static subspace (Eqs. 7, 8)
# ---------------------------------------------------------------------------


def subspace(chibar0: np.ndarray, n_eig: int):
    """Eigenpairs of the static v^1/2 chi0 v^1/2 with the largest |lambda|.

    The matrix is negative semidefinite, so these are the n_eig most negative
    eigenvalues; returned ascending with the matching eigenvector columns.
    Also returns the relative gap at the cut (lambda_{n_eig} - lambda_{n_eig-1})
    / |lambda_0| (zero-based), which decides whether the subspace is unique.
    """
    lam, vec = scipy.linalg.eigh(chibar0)
    n = chibar0.shape[0]
    gap = math.inf if n_eig >= n else (lam[n_eig] - lam[n_eig - 1]) / abs(lam[0])
    return lam[:n_eig].copy(), np.ascontiguousarray(vec[:, :n_eig]), gap


def project(w: np.ndarray, c_s: np.ndarray) -> np.ndarray:
    """W_s = W C_s  (Eq. 7, with the Coulomb factor folded into W)."""
    return w @ c_s


# ---------------------------------------------------------------------------
# Trace-log per frequency and quadrature (Eq. 1)
# ---------------------------------------------------------------------------


def _log1p_plus(y: np.ndarray) -> np.ndarray:
    """g(y) = ln(1 + y) - y, accurate to rounding also for small |y|.

    For |y| < 0.1 the Taylor series -sum_{k>=2} (-y)^k / k (60 terms, far
    past convergence); otherwise log1p(y) - y, which loses nothing there.
    """
    y = np.asarray(y, dtype=np.float64)
    out = np.log1p(y) - y
    small = np.abs(y) < 0.1
    ys = y[small]
    acc = np.zeros_like(ys)
    term = ys * ys
    for k in range(2, 62):
        acc += (term if k % 2 else -term) / k
        term = term * ys
    out[small] = acc
    return out


def trace_log(chis: np.ndarray, coupling: float = 1.0) -> float:
    """F = Tr ln(I - l chis) + l Tr chis = sum_k [ln(1 - l mu_k) + l mu_k]
    over the eigenvalues mu_k of the Hermitian chis (the definition of the
    trace of the logarithm), each term evaluated without cancellation."""
    mu = scipy.linalg.eigvalsh(chis)
    return float(np.sum(_log1p_plus(-coupling * mu)))


def trace_log_cholesky(chis: np.ndarray, coupling: float = 1.0) -> float:
    """ln det(I - l chis) + l Tr chis via a Cholesky factor (2 sum ln L_kk)."""
    n = chis.shape[0]
    b = np.eye(n) - coupling * chis
    low = np.linalg.cholesky(b)
    logdet = 2.0 * float(np.sum(np.log(np.real(np.diag(low)))))
    return logdet + coupling * float(np.real(np.trace(chis)))


def trace_log_lu(chis: np.ndarray, coupling: float = 1.0) -> float:
    """Same quantity from an LU factorization, as the paper describes."""
    n = chis.shape[0]
    lu, piv = scipy.linalg.lu_factor(np.eye(n) - coupling * chis)
    d = np.diag(lu)
    logdet = float(np.sum(np.log(np.abs(d))))
    return logdet + coupling * float(np.real(np.trace(chis)))


def quadrature(weights, integrand) -> float:
    """E_c = (1/2 pi) sum_j w_j F_j  (Eq. 1 with the integral discretized)."""
    return float(np.dot(np.asarray(weights), np.asarray(integrand))
                 / (2.0 * math.pi))


def gauss_legendre(n: int):
    """Gauss-Legendre nodes/weights on [-1, 1] by Golub-Welsch.

    The nodes are the eigenvalues of the Jacobi matrix with off-diagonal
    k / sqrt(4k^2 - 1); the weights are 2 (first eigenvector component)^2.
    """
    k = np.arange(1, n, dtype=np.float64)
    off = k / np.sqrt(4.0 * k * k - 1.0)
    x, v = scipy.linalg.eigh_tridiagonal(np.zeros(n), off)
    w = 2.0 * v[0, :] ** 2
    return x, w


def semi_infinite_rule(n: int, omega0: float = 1.0):
    """Gauss-Legendre mapped to [0, inf) by omega = omega0 (1+x)/(1-x)."""
    x, w = gauss_legendre(n)
    return omega0 * (1.0 + x) / (1.0 - x), 2.0 * omega0 * w / (1.0 - x) ** 2


# ---------------------------------------------------------------------------
# Whole pipeline
# ---------------------------------------------------------------------------


def pair_weights(eps, n_v, omega, occ=None) -> np.ndarray:
    """Delta_p(i omega) flattened over pairs p = v N_c + c.

    occ None: insulator (bands < n_v occupied); else pairs over V x C of
    band_sets(occ) with energy_factor_occ."""
    if occ is not None:
        return energy_factor_occ(eps, occ, omega).ravel()
    return energy_factor(eps[:n_v], eps[n_v:], omega).ravel()


def w_matrix(a, fft, miller_psi, coeff, n_v, ecut_chi, v_range=None,
             occ=None, truncation=None):
    """(W, Miller_chi) for all pairs (or valence bands v_range) via FFTs.

    occ None: V = bands < n_v, C = the rest; else the sets of band_sets."""
    mchi = chi_gvectors(a, ecut_chi)
    psi = orbitals_realspace(a, fft, miller_psi, coeff)
    if occ is None:
        vset, cset = np.arange(n_v), np.arange(n_v, coeff.shape[0])
    else:
        vset, cset = band_sets(occ)
    if v_range is not None:
        vset = vset[v_range[0]:v_range[1]]
    m = pair_matrix_fft(a, fft, psi[vset], psi[cset], mchi)
    return scaled_pair_matrix(a, m, mchi, truncation), mchi


def chi0_eq2_literal(a, miller_psi, coeff, eps, occ, miller_chi,
                     omega: float) -> np.ndarray:
    """Eq. (2) as printed, at q = 0 and one k-point (g = 1): the double sum
    over all ordered band pairs (n, n') with 2 (f_n' - f_n) and the complex
    denominator e_n' - e_n - i w, the matrix elements from the plane-wave
    convolution (no grid).  For time-reversal symmetric (real) orbitals this
    equals the pair form used everywhere else, transposed (reading of the
    exponent sign: e^{+iG.r} in Eq. 3 relabels G -> -G).  Small inputs only.
    """
    f = np.asarray(occ, dtype=np.float64)
    e = np.asarray(eps, dtype=np.float64)
    nb = coeff.shape[0]
    # x[n', n, G] = <psi_n'| e^{iG.r} |psi_n>
    x = pair_matrix_convolution(miller_psi, coeff, coeff, miller_chi)
    ng = x.shape[2]
    out = np.zeros((ng, ng), dtype=np.complex128)
    for n in range(nb):
        for n2 in range(nb):
            df = f[n2] - f[n]
            if df == 0.0:
                continue
            t = 2.0 * df / (e[n2] - e[n] - 1j * omega)
            out += t * np.outer(x[n2, n], np.conj(x[n2, n]))
    return out / cell_volume(a)


def trace_log_general(a_mat: np.ndarray, coupling: float = 1.0) -> float:
    """Tr ln(I - l A) + l Tr A for a matrix A that is similar to a Hermitian
    one (real spectrum), from its eigenvalues, term by term."""
    mu = np.real(np.linalg.eigvals(a_mat))
    return float(np.sum(_log1p_plus(-coupling * mu)))


def correlation_energy_chi0_basis(a, fft, miller_psi, coeff, energy, n_v,
                                  ecut_chi, n_eig, omega, weight, occ=None,
                                  truncation=None):
    """Static subspace from the eigenvectors of chi0 itself (Method, static
    subspace paragraph, read literally), step by step:

    1. M (Eq. 3) and chi0(0) = M^H Delta(0) M / Omega (Eq. 6).
    2. C_s = the n_eig eigenvectors of chi0(0) with the most negative
       eigenvalues.
    3. For every frequency chi0_s = (M C_s)^H Delta (M C_s) / Omega
       (Eqs. 7, 8) and the projected Coulomb kernel v_s = C_s^H v C_s, then
       F = Tr ln(1 - chi0_s v_s) + Tr chi0_s v_s from the eigenvalues of
       chi0_s v_s (C_s chi0_s C_s^H v restricted to the subspace).
    4. E_c = (1/2 pi) sum_j w_j F_j.
    """
    mchi = chi_gvectors(a, ecut_chi)
    psi = orbitals_realspace(a, fft, miller_psi, coeff)
    if occ is None:
        vset, cset = np.arange(n_v), np.arange(n_v, coeff.shape[0])
    else:
        vset, cset = band_sets(occ)
    m = pair_matrix_fft(a, fft, psi[vset], psi[cset], mchi)
    nv_, nc_, ng = m.shape
    mm = m.reshape(nv_ * nc_, ng)
    eps = np.asarray(energy)
    c0 = chibar(a, mm, pair_weights(eps, n_v, 0.0, occ))   # paper's chi0
    lam, vec = scipy.linalg.eigh(c0)
    c_s = vec[:, :n_eig]
    v = coulomb_kernel(a, mchi, truncation)
    v_s = (np.conj(c_s).T * v[None, :]) @ c_s
    ms = mm @ c_s
    f = np.empty(len(omega))
    for j, om in enumerate(omega):
        chis = chibar(a, ms, pair_weights(eps, n_v, float(om), occ))
        f[j] = trace_log_general(chis @ v_s)
    return dict(ec=quadrature(weight, f), integrand=f, eigval=lam[:n_eig],
                gap=(math.inf if n_eig >= ng else
                     (lam[n_eig] - lam[n_eig - 1]) / abs(lam[0])))


def epsilon_inverse(chis: np.ndarray) -> np.ndarray:
    """eps^-1 = (I - X)^-1 for the (projected) symmetrized matrix X
    (Implementation section, last paragraph: the factorization of the
    dielectric matrix 1 - chi0 v also yields eps^-1)."""
    n = chis.shape[0]
    return np.linalg.inv(np.eye(n) - chis)


def correlation_energy(a, fft, miller_psi, coeff, energy, n_v, ecut_chi,
                       n_eig, omega, weight, coupling=1.0, w=None, occ=None,
                       truncation=None):
    """Static-subspace RPA correlation energy, step by step.

    1. M by FFT (Eq. 3) and W = M v^1/2.
    2. chibar(0) (Eq. 6, symmetrized).
    3. C_s from its n_eig most negative eigenvectors.
    4. For every frequency: chibar_s = C_s^H chibar(i w) C_s computed as
       W_s^H diag(Delta) W_s / Omega (Eqs. 7, 8), then
       F = Tr ln(I - chibar_s) + Tr chibar_s from its eigenvalues (the
       Cholesky and LU forms of the paper's ln det agree with it, see
       trace_log_cholesky / trace_log_lu; the eigenvalue form has no
       rounding floor from cancelling ln det against the trace).
    5. E_c = (1/2 pi) sum_j w_j F_j.
    n_eig >= N_G means the full G basis (C_s = I).  occ: occupation factors
    (Eqs. 4-6), None for an insulator with n_v occupied bands.  truncation:
    None (bare Coulomb kernel) or "slab" (coulomb_slab).
    """
    if w is None:
        w, _ = w_matrix(a, fft, miller_psi, coeff, n_v, ecut_chi, occ=occ,
                        truncation=truncation)
    ng = w.shape[1]
    eps = np.asarray(energy)
    cb0 = chibar(a, w, pair_weights(eps, n_v, 0.0, occ))
    full = n_eig >= ng
    if full:
        lam = scipy.linalg.eigvalsh(cb0)
        ws, gap = w, math.inf
    else:
        lam, c_s, gap = subspace(cb0, n_eig)
        ws = project(w, c_s)
    f = np.empty(len(omega))
    chis_all = []
    for j, om in enumerate(omega):
        chis = chibar(a, ws, pair_weights(eps, n_v, float(om), occ))
        chis_all.append(chis)
        f[j] = trace_log(chis, coupling)
    ec = quadrature(weight, f)
    return dict(ec=ec, integrand=f, eigval=lam, gap=gap, chibar0=cb0,
                chis=chis_all)


# ---------------------------------------------------------------------------
# k-point sampling and q != 0 (Eqs. 1-3 with the sums over k and q)
# ---------------------------------------------------------------------------
#
# Orbitals at a k-point are psi_nk(r) = Omega^-1/2 sum_G c_nk(G) e^{i(k+G).r};
# their periodic parts u_nk(r) = Omega^-1/2 sum_G c_nk(G) e^{iG.r} are what
# orbitals_realspace returns for the coefficients of k.  With q on the mesh
# and k + q = k' + G0 (k' a mesh point, G0 a reciprocal lattice vector),
# u_{k+q}(r) = e^{-iG0.r} u_k'(r).
#
# Pair matrix, with the bra on the valence side as at q = 0 (reading of the
# exponent sign): P_vc,k(q; G) = int u*_vk u_c,k+q e^{iG.r} dr.  Eq. (3)'s
# element (bra at k + q) is M(G) = conj P(-G), so the paper's
# v(q+G)^1/2 chi0(q) v(q+G')^1/2 equals, at G -> -G and complex conjugated,
# the matrix built from P with v(G - q) = 4 pi / |G - q|^2 on the set
# {G : |G - q|^2 / 2 <= E_chi, G != q}: the same spectrum, F_j and E_c(q).
#
# Delta (reading 2 with k): the anti-resonant term of the pair (v at k,
# c at k + q) in Eq. (2) is the pair (c at k, v at k + q); for a k set closed
# under k -> -k with psi_{-k} = conj psi_k (time reversal) it equals the
# resonant term of (v at -k - q, c at -k), so
# chi0(q) = (1/Omega) sum_k g_k sum_vc conj(P) Delta P with
# Delta = -4 (e_c,k+q - e_vk) / ((e_c,k+q - e_vk)^2 + w^2) (insulators).


def chi_gvectors_q(a: float, ecut_chi: float, q) -> np.ndarray:
    """Miller indices G of the chi0 basis at q (fractional coordinates):
    |G - q|^2 / 2 <= ecut_chi, G != q.  Lexicographic in (n1, n2, n3)."""
    b = recip_unit(a)
    qf = np.asarray(q, dtype=np.float64)
    nmax = int(math.floor(math.sqrt(2.0 * ecut_chi) / b + np.max(np.abs(qf)))) + 1
    out = []
    for n1 in range(-nmax, nmax + 1):
        for n2 in range(-nmax, nmax + 1):
            for n3 in range(-nmax, nmax + 1):
                d = np.array([n1, n2, n3], dtype=np.float64) - qf
                d2 = float(d @ d)
                if d2 == 0.0:
                    continue
                if 0.5 * b * b * d2 <= ecut_chi:
                    out.append((n1, n2, n3))
    return np.array(out, dtype=np.int64).reshape(-1, 3)


def coulomb_q(a: float, miller: np.ndarray, q) -> np.ndarray:
    """v(G - q) = 4 pi / |G - q|^2 for the chi0 basis at q."""
    b = recip_unit(a)
    d = np.asarray(miller, dtype=np.float64) - np.asarray(q, dtype=np.float64)
    return 4.0 * math.pi / (b * b * np.sum(d * d, axis=1))


def pair_matrix_kq(a, fft, u_v, u_c, g0, miller_chi) -> np.ndarray:
    """P_vc(G) = (Omega / N) sum_j conj(u_v(r_j)) u_c(r_j) e^{-iG0.r_j}
    e^{iG.r_j}: u_v the periodic parts at k, u_c those at k' with
    k + q = k' + G0.  Returns [v, c, G]."""
    n1, n2, n3 = fft
    m = np.asarray(miller_chi) - np.asarray(g0)[None, :]
    out = np.empty((u_v.shape[0], u_c.shape[0], m.shape[0]), dtype=np.complex128)
    omega = cell_volume(a)
    for iv in range(u_v.shape[0]):
        rho = np.conj(u_v[iv])[None] * u_c
        f = scipy.fft.ifftn(rho, axes=(1, 2, 3), workers=-1)
        out[iv] = omega * f[:, m[:, 0] % n1, m[:, 1] % n2, m[:, 2] % n3]
    return out


def correlation_energy_q(a, fft, kpoints, q, kq, g0, ecut_chi, n_eig, omega,
                         weight):
    """E_c(q) of Eq. (1) for one q of a k mesh, step by step (insulators).

    kpoints: list of dicts with keys miller, coeff, energy, n_v, weight (g_k).
    kq[i], g0[i]: k_i + q = k_kq[i] + g0[i].  Steps as in correlation_energy,
    with the pair rows of every k stacked (weights g_k folded into Delta).
    Returns dict(ec, integrand, eigval, gap, chibar0, chis).
    """
    mchi = chi_gvectors_q(a, ecut_chi, q)
    sv = np.sqrt(coulomb_q(a, mchi, q))
    us = [orbitals_realspace(a, fft, k["miller"], k["coeff"]) for k in kpoints]
    ws, des, gks = [], [], []
    for i, k in enumerate(kpoints):
        kp = kpoints[kq[i]]
        nv = k["n_v"]
        p = pair_matrix_kq(a, fft, us[i][:nv], us[kq[i]][kp["n_v"]:], g0[i], mchi)
        ws.append(p.reshape(-1, len(mchi)) * sv[None, :])
        de = kp["energy"][kp["n_v"]:][None, :] - k["energy"][:nv][:, None]
        des.append(de.ravel())
        gks.append(np.full(de.size, float(k["weight"])))
    w = np.concatenate(ws)
    de = np.concatenate(des)
    gk = np.concatenate(gks)

    def delta(om):
        return gk * (-4.0 * de / (de * de + om * om))
    ng = len(mchi)
    cb0 = chibar(a, w, delta(0.0))
    if n_eig >= ng:
        lam = scipy.linalg.eigvalsh(cb0)
        wsub, gap = w, math.inf
    else:
        lam, c_s, gap = subspace(cb0, n_eig)
        wsub = project(w, c_s)
    f = np.empty(len(omega))
    chis_all = []
    for j, om in enumerate(omega):
        chis = chibar(a, wsub, delta(float(om)))
        chis_all.append(chis)
        f[j] = trace_log(chis)
    return dict(ec=quadrature(weight, f), integrand=f, eigval=lam, gap=gap,
                chibar0=cb0, chis=chis_all, miller_chi=mchi)


def chi0_q_eq2_literal(a, kpoints, q, kq, g0, miller_chi_paper, omega):
    """Eq. (2) as printed at q: sum over k and all ordered band pairs
    (n at k, n' at k + q) of 2 g_k (f_n',k+q - f_nk) M(G) conj M(G') /
    (e_n',k+q - e_nk - i w) with Eq. (3)'s M = <psi_n',k+q| e^{i(q+G).r}
    |psi_nk>, from plane-wave coefficients (no grid): the coefficient of
    the Bloch function at k + q is c_k'(G + G0).  Occupations 1 below n_v,
    0 above.  Small inputs only; returns chi0_GG'(q) over miller_chi_paper
    (the G of q + G).  Since M(G) = conj P(-G), this equals the pair form
    built from P at (-G, -G') when the k set is time-reversal symmetric."""
    mc = np.asarray(miller_chi_paper, dtype=np.int64)
    out = np.zeros((len(mc), len(mc)), dtype=np.complex128)
    for i, k in enumerate(kpoints):
        kp = kpoints[kq[i]]
        # <psi_n',k+q| e^{i(q+G).r} |psi_nk> = sum_G1 conj(c_n',k+q(G1)) c_nk(G1 - G)
        # with the k+q coefficients c_k'(. + G0)
        idx_k = {tuple(int(x) for x in m): j for j, m in enumerate(k["miller"])}
        mkp = np.asarray(kp["miller"], dtype=np.int64) - np.asarray(g0[i])[None, :]
        nb, nbp = k["coeff"].shape[0], kp["coeff"].shape[0]
        x = np.zeros((nbp, nb, len(mc)), dtype=np.complex128)
        for ig, g in enumerate(mc):
            src, dst = [], []
            for j1, g1 in enumerate(mkp):
                j = idx_k.get((int(g1[0] - g[0]), int(g1[1] - g[1]), int(g1[2] - g[2])))
                if j is not None:
                    src.append(j1)
                    dst.append(j)
            if src:
                x[:, :, ig] = np.conj(kp["coeff"][:, src]) @ k["coeff"][:, dst].T
        f_k = (np.arange(nb) < k["n_v"]).astype(float)
        f_kp = (np.arange(nbp) < kp["n_v"]).astype(float)
        for n in range(nb):
            for n2 in range(nbp):
                df = f_kp[n2] - f_k[n]
                if df == 0.0:
                    continue
                t = 2.0 * k["weight"] * df / (kp["energy"][n2] - k["energy"][n] - 1j * omega)
                out += t * np.outer(x[n2, n], np.conj(x[n2, n]))
    return out / cell_volume(a)


# ---------------------------------------------------------------------------
# Closed forms used to pin the above
# ---------------------------------------------------------------------------


def plasmon_ec(a, w, d_eps) -> float:
    """Exact-frequency full-basis RPA E_c from the pair-space plasmon formula.

    With D = diag(de_p) and Kt = W W^H / Omega (pairs x pairs),
    E_c = 1/2 Tr[(D^2 + 4 D^1/2 Kt D^1/2)^1/2] - 1/2 Tr D - Tr Kt.
    It follows from det(I - A B) = det(I - B A) and the integral
    int_0^inf dw/(2 pi) ln((x^2 + w^2)/(y^2 + w^2)) = (x - y)/2.
    """
    d = np.asarray(d_eps, dtype=np.float64)
    kt = w @ np.conj(w).T / cell_volume(a)
    sd = np.sqrt(d)
    mat = np.diag(d * d) + 4.0 * sd[:, None] * kt * sd[None, :]
    ev = scipy.linalg.eigvalsh(mat)
    return float(0.5 * np.sum(np.sqrt(ev)) - 0.5 * np.sum(d)
                 - np.real(np.trace(kt)))


def direct_mp2(a, w, d_eps) -> float:
    """Second-order (coupling^2) term of E_c: -2 sum_pq |Kt_pq|^2/(d_p + d_q)."""
    d = np.asarray(d_eps, dtype=np.float64)
    kt = w @ np.conj(w).T / cell_volume(a)
    return float(-2.0 * np.sum(np.abs(kt) ** 2 / (d[:, None] + d[None, :])))


def second_order_quadrature(a, w, eps, n_v, omega, weight) -> float:
    """-(1/4 pi) sum_j w_j Tr[chibar(i w_j)^2], the lambda^2 coefficient."""
    tot = 0.0
    for om, wt in zip(omega, weight):
        cb = chibar(a, w, pair_weights(np.asarray(eps), n_v, float(om)))
        tot += wt * float(np.real(np.sum(cb * cb.T)))
    return -tot / (4.0 * math.pi)
