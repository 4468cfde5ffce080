"""Two-photon observables from two-channel transfer coefficients (test infrastructure only).

Transfer coefficients are ordered ``T = (T_a1, T_a2, T_b1, T_b2)``: detector
a (position r1, polarisation e_a) or b, input channel 1 or 2 (the paper's
two-channel transfer relation, eqs. field_transfer1/2).

* g2 (eq. 10): w1 w2 |T_a1 T_b2 + T_a2 T_b1|^2 /
  ((w1|T_a1|^2 + w2|T_a2|^2)(w1|T_b1|^2 + w2|T_b2|^2)).
* Coincidences (eqs. 18-22) with path amplitudes A_dir = T_a1 T_b2,
  A_ex = T_a2 T_b1 (eq. path_amplitudes) and the baseband Gaussian overlap
  h(tau) = exp(-tau^2 / (2 sigma^2)) (eq. h_gauss without the carrier, whose
  literal inclusion would suppress the cross term by exp(-w0^2 sigma^2)):
  Nc(dtau) = sigma sqrt(pi) [|A_dir|^2 + |A_ex|^2 + 2 Re(A_dir A_ex*) c(dtau)],
  c = exp(-dtau^2 / sigma^2), K = 1.
  Normalisation R1: D_c = sigma sqrt(pi) (|A_dir|^2 + |A_ex|^2), so that
  Nc~ -> 1 at large delay.  R2: D_c = sigma sqrt(pi) G1_a G1_b (product of
  marginal intensities), so that Nc~(0) = g2 and single-path zeros stay zero.
  Channel weights w_j (the sqrt(omega_kj) factors of the field operators,
  eqs. 8-9) multiply every transfer coefficient of channel j by sqrt(w_j)
  before any of the above, exactly as they enter g2 (eq. 10).
* Classical comparison (eq. 27): P2 = |T_a1 + T_a2|^2 |T_b1 + T_b2|^2.
"""

from __future__ import annotations

import itertools

import numpy as np

SQRT_PI = np.sqrt(np.pi)


def g2(T, omega=(1.0, 1.0)):
    """Normalised second-order correlation of two populated channels (eq. 10).
    NaN when a detector is dark (0/0)."""
    Ta1, Ta2, Tb1, Tb2 = (complex(v) for v in T)
    w1, w2 = omega
    num = w1 * w2 * abs(Ta1 * Tb2 + Ta2 * Tb1) ** 2
    den = (w1 * abs(Ta1) ** 2 + w2 * abs(Ta2) ** 2) * (w1 * abs(Tb1) ** 2 + w2 * abs(Tb2) ** 2)
    return num / den if den > 0 else float("nan")


def classical_p2(T):
    """Classical fourth-order correlation (eq. 27): intensity product
    |E(r1)|^2 |E(r2)|^2 of the coherent superposition E = E_k1 + E_k2 of the
    two channels' responses, projected on the detectors."""
    Ta1, Ta2, Tb1, Tb2 = (complex(v) for v in T)
    return abs(Ta1 + Ta2) ** 2 * abs(Tb1 + Tb2) ** 2


def g2_fock(T, omega=(1.0, 1.0), nmax=2):
    """Brute-force g2 from the normally ordered expectation sum (eq. 11) in a
    truncated two-mode Fock space with input |1_1, 1_2>.  Mode amplitudes carry
    sqrt(w_j) (eqs. 8-9).  Independent of the compact form above."""
    d = nmax + 1
    a = np.diag(np.sqrt(np.arange(1, d)), 1)  # single-mode annihilation
    I = np.eye(d)
    ops = [np.kron(a, I), np.kron(I, a)]
    vac = np.zeros(d * d)
    vac[0] = 1.0
    psi = ops[0].T @ ops[1].T @ vac  # a1^dag a2^dag |0>
    Ta = np.array([T[0], T[1]], complex) * np.sqrt(omega)
    Tb = np.array([T[2], T[3]], complex) * np.sqrt(omega)
    num = 0j
    for m, n, p, q in itertools.product(range(2), repeat=4):
        ex = psi @ (ops[m].T @ ops[n].T @ ops[p] @ ops[q] @ psi)
        num += np.conj(Ta[m]) * np.conj(Tb[n]) * Tb[p] * Ta[q] * ex
    Ga = sum(np.conj(Ta[m]) * Ta[q] * (psi @ (ops[m].T @ ops[q] @ psi)) for m in range(2) for q in range(2))
    Gb = sum(np.conj(Tb[n]) * Tb[p] * (psi @ (ops[n].T @ ops[p] @ psi)) for n in range(2) for p in range(2))
    den = (Ga * Gb).real
    return float(num.real / den) if den > 0 else float("nan")


def path_amplitudes(T):
    """A_dir = T_a1 T_b2, A_ex = T_a2 T_b1 (eq. path_amplitudes)."""
    return complex(T[0]) * complex(T[3]), complex(T[1]) * complex(T[2])


def weighted(T, omega=(1.0, 1.0)):
    """Transfer coefficients with the channel weights of eqs. 8-9 folded in:
    T_aj, T_bj -> sqrt(w_j) T_aj, sqrt(w_j) T_bj."""
    s1, s2 = np.sqrt(omega[0]), np.sqrt(omega[1])
    return (s1 * complex(T[0]), s2 * complex(T[1]), s1 * complex(T[2]), s2 * complex(T[3]))


def coincidence(T, sigma, dtau, norm="R1", omega=(1.0, 1.0)):
    """Closed-form coincidence number.  Returns (Nc_raw, Nc_norm) arrays over
    dtau (eqs. 18-22, K = 1, baseband Gaussian wavepackets), channel weights
    folded into the transfer coefficients (eqs. 8-9)."""
    dtau = np.asarray(dtau, float)
    T = weighted(T, omega)
    Ad, Ae = path_amplitudes(T)
    c = np.exp(-(dtau**2) / sigma**2)
    raw = sigma * SQRT_PI * (abs(Ad) ** 2 + abs(Ae) ** 2 + 2.0 * np.real(Ad * np.conj(Ae)) * c)
    if norm == "R1":
        D = sigma * SQRT_PI * (abs(Ad) ** 2 + abs(Ae) ** 2)
    elif norm == "R2":
        Ga = abs(T[0]) ** 2 + abs(T[1]) ** 2
        Gb = abs(T[2]) ** 2 + abs(T[3]) ** 2
        D = sigma * SQRT_PI * Ga * Gb
    else:
        raise ValueError(norm)
    nrm = raw / D if D > 0 else np.full_like(raw, np.nan)
    return raw, nrm


def coincidence_quadrature(T, sigma, dtau, n=4001, span=12.0, omega=(1.0, 1.0)):
    """Raw Nc by direct tau quadrature of the scattering correlation
    (eq. G2_scatter) with baseband h(tau) = exp(-tau^2/(2 sigma^2)); trapezoid
    rule on a wide uniform grid (spectrally accurate for Gaussians)."""
    Ad, Ae = path_amplitudes(weighted(T, omega))
    out = []
    for dt in np.atleast_1d(dtau):
        lo, hi = min(0.0, 2 * dt) - span * sigma, max(0.0, 2 * dt) + span * sigma
        tau = np.linspace(lo, hi, n)
        h1 = np.exp(-(tau**2) / (2 * sigma**2))
        h2 = np.exp(-((2 * dt - tau) ** 2) / (2 * sigma**2))
        G2 = (abs(Ad) ** 2 * np.abs(h1) ** 2 + abs(Ae) ** 2 * np.abs(h2) ** 2
              + Ad * np.conj(Ae) * h1 * np.conj(h2) + np.conj(Ad) * Ae * np.conj(h1) * h2)
        out.append(np.trapezoid(G2.real, tau))
    return np.asarray(out)


def beam_splitter_T(Tbs, Rbs):
    """Transfer coefficients of the phase-asymmetric beam splitter (eqs. 15-16
    at zero delay): T_a1 = sqrt(T), T_a2 = i sqrt(R), T_b1 = i sqrt(R), T_b2 = sqrt(T)."""
    return (np.sqrt(Tbs), 1j * np.sqrt(Rbs), 1j * np.sqrt(Rbs), np.sqrt(Tbs))


def beam_splitter_nc_quadrature(Tbs, Rbs, sigma, dtau, n=4001, span=12.0):
    """Raw Nc of the textbook beam-splitter correlation (eq. 17, K = 1) by
    tau quadrature, baseband h."""
    out = []
    for dt in np.atleast_1d(dtau):
        lo, hi = min(0.0, 2 * dt) - span * sigma, max(0.0, 2 * dt) + span * sigma
        tau = np.linspace(lo, hi, n)
        h1 = np.exp(-(tau**2) / (2 * sigma**2))
        h2 = np.exp(-((2 * dt - tau) ** 2) / (2 * sigma**2))
        G2 = Tbs**2 * h1**2 + Rbs**2 * h2**2 - 2 * Rbs * Tbs * h1 * h2
        out.append(np.trapezoid(G2, tau))
    return np.asarray(out)
