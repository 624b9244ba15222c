"""Pins of the imaginary-axis correlation self-energy oracle
(oracle/sigc_oracle.py) against what Eq.(sigci), the reading of its
integration weights and linear algebra fix: hand-derived weights, adaptive
numerical integration of the interpolant, the exact integral of a Lorentzian
W^c within the interpolation error bound, the limits dE -> 0 and dE -> inf,
exact rational arithmetic and explicit loops for the contraction, and
structural identities (Hermiticity and sign for degenerate states, phases,
permutations, additivity)."""
import math
from fractions import Fraction

import numpy as np

U = np.finfo(np.float64).eps / 2


def _close(a, b, tol):
    a = np.asarray(a)
    b = np.asarray(b)
    return np.max(np.abs(a - b)) <= tol * max(1.0, np.max(np.abs(b)))


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) /
                 max(np.linalg.norm(np.asarray(b)), 1e-300))


# ----------------------------------------------------------------- weights
def pin_weights_hand(orc):
    """Closed forms worked out by hand from the reading:
    mesh {0, 1}, dE = 1:  X interpolated as (1-w) X0 + w X1 on [0, 1] and
    X1 / w^2 beyond, so
      w0 = (1/pi) int_0^1 (1-w)/(1+w^2) dw = 1/4 - ln2/(2 pi),
      w1 = (1/pi)[int_0^1 w/(1+w^2) dw + int_1^inf dw/(w^2 (1+w^2))]
         = ln2/(2 pi) + 1/pi - 1/4;
    mesh {1/2}, dE = 1: constant on [0, 1/2], X0/(4 w^2) beyond:
      w0 = (1/pi)[atan(1/2) + 1/2 - atan(2)/4]."""
    fails = []
    got = orc.ag_weights(1.0, [0.0, 1.0])
    ref = [0.25 - math.log(2) / (2 * math.pi), math.log(2) / (2 * math.pi) + 1 / math.pi - 0.25]
    if not _close(got, ref, 4 * U):
        fails.append(f"hand weights mesh {{0,1}}: {got} vs {ref}")
    if not _close(orc.ag_weights(-1.0, [0.0, 1.0]), [-x for x in ref], 4 * U):
        fails.append("hand weights dE = -1")
    got = orc.ag_weights(1.0, [0.5])
    ref = [(math.atan(0.5) + 0.5 - math.atan(2.0) / 4) / math.pi]
    if not _close(got, ref, 4 * U):
        fails.append(f"hand weights mesh {{1/2}}: {got} vs {ref}")
    return fails


def _interp_integral(mesh, x, d):
    """(1/pi) int_0^inf X(w) d/(d^2+w^2) dw for the interpolant of the
    reading, by adaptive quadrature (scipy), piece by piece."""
    from scipy.integrate import quad
    mesh = list(mesh)

    def f(w, a, xa, b, xb):
        return (xa + (xb - xa) * (w - a) / (b - a)) * d / (d * d + w * w)

    tot = 0.0
    if mesh[0] > 0:
        tot += quad(lambda w: x[0] * d / (d * d + w * w), 0.0, mesh[0],
                    epsabs=0, epsrel=1e-13, limit=200)[0]
    for j in range(len(mesh) - 1):
        tot += quad(f, mesh[j], mesh[j + 1], args=(mesh[j], x[j], mesh[j + 1], x[j + 1]),
                    epsabs=0, epsrel=1e-13, limit=200)[0]
    c = mesh[-1]
    tot += quad(lambda w: x[-1] * (c / w) ** 2 * d / (d * d + w * w), c, np.inf,
                epsabs=0, epsrel=1e-13, limit=200)[0]
    return tot / math.pi


def pin_weights_quadrature(orc):
    """sum_i w_i X_i equals the adaptive-quadrature integral of the
    interpolant times the Lorentzian, for random meshes, nodes and dE."""
    import warnings
    fails = []
    rng = np.random.default_rng(21)
    for trial in range(12):
        n = int(rng.integers(1, 9))
        mesh = np.cumsum(rng.uniform(0.05, 2.0, n))
        if trial % 3 == 0:
            mesh = mesh - mesh[0]                     # first node at w = 0
        if n == 1 and mesh[0] == 0:
            mesh = mesh + 0.3
        x = rng.uniform(-1, 1, n)
        d = float(rng.choice([-1, 1]) * 10 ** rng.uniform(-2.5, 1.5))
        with warnings.catch_warnings():
            warnings.simplefilter("ignore")
            ref = _interp_integral(mesh, x, d)
        got = float(orc.ag_weights(d, mesh) @ x)
        if abs(got - ref) > 1e-10 * max(1.0, abs(ref)):
            fails.append(f"quadrature trial {trial}: {got} vs {ref} (d={d}, n={n})")
    return fails


def pin_weights_lorentzian(orc):
    """X(w) = O^2/(O^2 + w^2) (a single-plasmon-like W^c): the exact integral
    is sign(dE) O / (2 (|dE| + O)).  On uniform meshes of step h up to w_max
    the interpolant differs from X by at most h^2 max|X''| / 8 = h^2/(4 O^2)
    on the mesh and by at most O^2/w_max^2 beyond it (relative), while the
    Lorentzian integrates to at most 1/2; the error must respect that bound
    and fall by about 4 when h halves."""
    fails = []
    om = 0.7
    for d in (0.01, 0.3, 2.0, -0.3):
        exact = math.copysign(om / (2 * (abs(d) + om)), d)
        errs = []
        for n in (101, 201):
            wmax = 40.0
            mesh = np.linspace(0.0, wmax, n)
            h = mesh[1]
            x = om * om / (om * om + mesh ** 2)
            err = abs(float(orc.ag_weights(d, mesh) @ x) - exact)
            bound = 0.5 * (h * h / (4 * om * om) + om * om / wmax ** 2)
            if err > bound:
                fails.append(f"Lorentzian d={d} n={n}: error {err} above bound {bound}")
            errs.append(err)
        if not (errs[1] < errs[0]):
            fails.append(f"Lorentzian d={d}: no convergence {errs}")
    return fails


def pin_weights_limits(orc):
    """dE -> 0+: the Lorentzian tends to delta(w)/2, so the first node (at
    w = 0) takes 1/2 and the others 0; dE = 0 gives 0; odd in dE; scale
    invariant (dE and the mesh scaled by 2); dE -> inf: w_i -> (int of node
    i's basis function) / (pi dE), i.e. w_0 h_0/2 + ..., the tail adding
    w_{n-1} (its integral of (c/w)^2 beyond c is c; the tail converges only
    as 1 - O(c/dE), hence the large dE)."""
    fails = []
    mesh = np.array([0.0, 0.2, 0.7, 1.5, 4.0])
    w = orc.ag_weights(1e-13, mesh)
    if not _close(w, [0.5, 0, 0, 0, 0], 1e-11):
        fails.append(f"dE -> 0+: {w}")
    if np.any(orc.ag_weights(0.0, mesh) != 0):
        fails.append("dE = 0 not zero")
    for d in (0.03, 1.7, 55.0):
        if not np.array_equal(orc.ag_weights(-d, mesh), -orc.ag_weights(d, mesh)):
            fails.append(f"not odd at {d}")
        if not np.array_equal(orc.ag_weights(2 * d, 2 * mesh), orc.ag_weights(d, mesh)):
            fails.append(f"not scale invariant at {d}")
    d = 1e11
    h = np.diff(mesh)
    basis = np.zeros(len(mesh))
    basis[:-1] += h / 2
    basis[1:] += h / 2
    basis[-1] += mesh[-1]
    if not _close(orc.ag_weights(d, mesh) * math.pi * d, basis, 1e-9):
        fails.append(f"dE -> inf: {orc.ag_weights(d, mesh) * math.pi * d} vs {basis}")
    return fails


# ------------------------------------------------------------- contraction
def _rand_block(rng, nall, npb, nqp, nom, scale=1.0):
    z = (rng.standard_normal((nall, npb, nqp)) + 1j * rng.standard_normal((nall, npb, nqp))) * scale
    a = rng.standard_normal((nom, npb, npb)) + 1j * rng.standard_normal((nom, npb, npb))
    wc = -(a @ np.conj(np.transpose(a, (0, 2, 1)))) / npb       # Hermitian, <= 0
    return z, wc


def pin_contract_exact_and_brute(orc):
    """Small-integer Z and W, dyadic weights and w_k: exact rational
    contraction = the numpy contraction; explicit loops = the reference
    with the weights of the reading (two blocks, every dimension > 1)."""
    fails = []
    rng = np.random.default_rng(5)
    nqp, nom = 3, 2
    ex_in, np_in = [], []
    for nall, npb, wk in ((2, 3, Fraction(1, 2)), (3, 2, Fraction(3, 8))):
        zr = rng.integers(-3, 4, (nall, npb, nqp))
        zi = rng.integers(-3, 4, (nall, npb, nqp))
        wr = rng.integers(-4, 5, (nom, npb, npb))
        wi = rng.integers(-4, 5, (nom, npb, npb))
        wt = rng.integers(-8, 9, (nall, nqp, nom))
        ex_in.append(([[[(Fraction(int(zr[a, m, n])), Fraction(int(zi[a, m, n])))
                         for n in range(nqp)] for m in range(npb)] for a in range(nall)],
                      [[[(Fraction(int(wr[i, m, v])), Fraction(int(wi[i, m, v])))
                         for v in range(npb)] for m in range(npb)] for i in range(nom)],
                      [[[Fraction(int(wt[a, n, i]), 16) for i in range(nom)]
                        for n in range(nqp)] for a in range(nall)], wk))
        np_in.append((zr + 1j * zi, wr + 1j * wi, wt / 16.0, float(wk)))
    ex = orc.sigc_contract_exact(ex_in, nqp)
    ex = np.array([[float(r) + 1j * float(i) for r, i in row] for row in ex])
    if not _close(orc.sigc_contract(np_in, nqp), ex, 1e-15):
        fails.append("numpy contraction != exact rational")
    mesh = [0.0, 0.4, 1.3]
    eps_qp = np.array([-0.5, 0.1, 0.9])
    blocks = []
    for nall, npb in ((2, 3), (3, 2)):
        z, wc = _rand_block(rng, nall, npb, 3, len(mesh))
        blocks.append((z, wc, rng.uniform(-1, 1, nall), 0.25))
    if not _close(orc.sigc_brute(blocks, eps_qp, mesh), orc.sigc_ref(blocks, eps_qp, mesh), 1e-13):
        fails.append("brute loops != reference")
    if not _close(orc.sigc_rows(blocks, eps_qp, mesh, [2, 0]),
                  orc.sigc_ref(blocks, eps_qp, mesh)[[2, 0]], 1e-14):
        fails.append("row sampler != reference")
    ent = [(0, 2), (1, 1), (2, 0)]
    sel = [(z[:, :, [0, 1, 2]], [0, 1, 2], wc, em, wk) for z, wc, em, wk in blocks]
    full = orc.sigc_ref(blocks, eps_qp, mesh)
    if not _close(orc.sigc_entries(sel, eps_qp, mesh, ent), [full[n, m] for n, m in ent], 1e-14):
        fails.append("entry sampler != reference")
    return fails


def pin_single_state(orc):
    """One intermediate state, one product-basis function: the sums
    collapse to I[n][m] = -w_k sum_i w_i(eps_n - e') W_i conj(z_n) z_m; the
    weight follows the row n (I[m][n] uses eps_m)."""
    fails = []
    mesh = [0.0, 0.5, 2.0]
    z = np.array([[[1 + 2j, -0.5 + 1j, 0.25 - 0.75j]]])
    wc = np.array([[[-1.0 + 0j]], [[-0.6 + 0j]], [[-0.1 + 0j]]])
    eps_qp = np.array([-0.4, 0.3, 1.1])
    e1 = 0.05
    got = orc.sigc_ref([(z, wc, np.array([e1]), 0.5)], eps_qp, mesh)
    ref = np.zeros((3, 3), complex)
    for n in range(3):
        wt = orc.ag_weights(float(eps_qp[n] - e1), mesh)
        for m in range(3):
            ref[n, m] = -0.5 * sum(wt[i] * wc[i, 0, 0] for i in range(3)) * np.conj(z[0, 0, n]) * z[0, 0, m]
    if not _close(got, ref, 1e-15):
        fails.append("single-state closed form")
    return fails


def pin_structure(orc):
    """Degenerate quasiparticle energies make I Hermitian; with W <= 0 and
    every intermediate state below them the weights are >= 0 and I >= 0.
    Additivity over blocks, permutation of n' (energies with it), a phase
    per n' leave I unchanged; a phase e^{i t_n} per state n gives
    I[n][m] e^{-i t_n} e^{i t_m}; I is linear in W."""
    fails = []
    rng = np.random.default_rng(8)
    mesh = [0.0, 0.3, 1.0, 3.0]
    nqp = 4
    z, wc = _rand_block(rng, 3, 5, nqp, len(mesh))
    deg = np.full(nqp, 0.7)
    i_deg = orc.sigc_ref([(z, wc, np.array([-0.5, 0.1, 0.3]), 1.0)], deg, mesh)
    if not _close(i_deg, i_deg.conj().T, 1e-14):
        fails.append("degenerate states: not Hermitian")
    ev = np.linalg.eigvalsh((i_deg + i_deg.conj().T) / 2)
    if ev.min() < -1e-13 * abs(ev).max():
        fails.append(f"degenerate states below: not >= 0 ({ev.min()})")

    eps_qp = np.array([-0.6, -0.1, 0.4, 1.2])
    em1 = np.array([-0.5, 0.1, 0.3])
    z2, wc2 = _rand_block(rng, 2, 5, nqp, len(mesh))
    em2 = np.array([-0.2, 0.8])
    b1 = (z, wc, em1, 0.5)
    b2 = (z2, wc2, em2, 0.25)
    both = orc.sigc_ref([b1, b2], eps_qp, mesh)
    sep = orc.sigc_ref([b1], eps_qp, mesh) + orc.sigc_ref([b2], eps_qp, mesh)
    if not _close(both, sep, 1e-14):
        fails.append("not additive over blocks")
    perm = rng.permutation(3)
    if not _close(orc.sigc_ref([(z[perm], wc, em1[perm], 0.5)], eps_qp, mesh),
                  orc.sigc_ref([b1], eps_qp, mesh), 1e-14):
        fails.append("n' permutation changes I")
    ph = np.exp(1j * rng.uniform(0, 2 * np.pi, 3))[:, None, None]
    if not _close(orc.sigc_ref([(z * ph, wc, em1, 0.5)], eps_qp, mesh),
                  orc.sigc_ref([b1], eps_qp, mesh), 1e-14):
        fails.append("phase per n' changes I")
    t = rng.uniform(0, 2 * np.pi, nqp)
    got = orc.sigc_ref([(z * np.exp(1j * t)[None, None, :], wc, em1, 0.5)], eps_qp, mesh)
    ref = orc.sigc_ref([b1], eps_qp, mesh) * np.exp(-1j * t)[:, None] * np.exp(1j * t)[None, :]
    if not _close(got, ref, 1e-14):
        fails.append("phase per state n: wrong covariance")
    if not _close(orc.sigc_ref([(z, 3 * wc, em1, 0.5)], eps_qp, mesh),
                  3 * orc.sigc_ref([b1], eps_qp, mesh), 1e-14):
        fails.append("not linear in W")
    return fails


def pin_w_orientation(orc):
    """A W with a single entry W_i[mu][nu] = 1 (mu != nu) couples
    conj(Z[mu][n]) on the left to Z[nu][m] on the right only."""
    fails = []
    mesh = [0.0, 1.0]
    z = np.zeros((1, 2, 2), complex)
    z[0, 0, 0] = 1.0          # Z[mu=0][n=0]
    z[0, 1, 1] = 1j           # Z[mu=1][n=1]
    wc = np.zeros((2, 2, 2), complex)
    wc[:, 0, 1] = 1.0         # W[mu=0][nu=1]
    eps_qp = np.array([0.5, 0.5])
    got = orc.sigc_ref([(z, wc, np.array([0.0]), 1.0)], eps_qp, mesh)
    wsum = float(orc.ag_weights(0.5, mesh).sum())
    ref = np.zeros((2, 2), complex)
    ref[0, 1] = -wsum * np.conj(1.0) * 1.0 * 1j      # conj(Z[0][0]) W[0][1] Z[1][1]
    if not _close(got, ref, 1e-15):
        fails.append(f"W orientation: {got}")
    return fails


PINS = [pin_weights_hand, pin_weights_quadrature, pin_weights_lorentzian, pin_weights_limits,
        pin_contract_exact_and_brute, pin_single_state, pin_structure, pin_w_orientation]


def run_all(orc):
    return {p.__name__: p(orc) for p in PINS}
