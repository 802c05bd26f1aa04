"""Closed forms printed in the paper, transcribed on the test side to pin the oracle.

Each function cites the equation it restates.  Nothing here is shared with the oracle or the
GPU library; an error in the oracle's own transcription shows up as a disagreement here.
"""
import math

SQ6PI = math.sqrt(6.0 / math.pi)


def tau_s_of_kn(kn, h):
    """Eq. (tKnrela)."""
    return 0.5 + SQ6PI * kn * h


def l1_poiseuille(sigma=1.0):
    """Sec. IV: L1 = (2 - sigma)(1 - 0.1817 sigma)/sigma."""
    return (2.0 - sigma) * (1.0 - 0.1817 * sigma) / sigma


def l2_poiseuille(l1):
    """Sec. IV: L2 = 1/pi + L1^2/2."""
    return 1.0 / math.pi + l1 * l1 / 2.0


def near_wall_coeffs(r, l, g, ts, tq):
    """Eqs. (NumerSana)-(CoeC): u_1 = A u_0 + B a dt + C u_w (label quirk: CoeAB holds A and C)."""
    den = (1 + l) * (1 - r) * ts + 2 * r * g
    A = ((1 + l) * (1 - r) * ts + 2 * r * (1 + g)) / den
    C = -2 * r / den
    B = ((1 + r + l - l * r) * (1 + 4 * tq - 8 * ts - 8 * tq * ts)
         + 12 * r * ((2 * g - l) * (2 * ts - 1) + (1 - 2 * g) * ts)) / (2 * den * (2 * ts - 1))
    return A, B, C


def near_wall_A_wall_reading(r, l, g, ts):
    """A of the steady near-wall relation when the diffuse equilibrium takes the wall velocity
    (literal reading of Eq. (EqNewBDSC)); derived by repeating the analysis of Sec. III.B with
    f^eq(rho, u_w) in place of f^eq(rho, u_0): the diffuse part then adds (1+l)(1-r) to the
    numerator.  Under that reading C = 1 - A and B is unchanged."""
    den = (1 + l) * (1 - r) * ts + 2 * r * g
    return ((1 + l) * (1 - r) * (ts + 1) + 2 * r * (1 + g)) / den


def slip_eqmislip(r, l, g, ts, tq, h):
    """Eq. (EqMiSlip): dimensionless slip U_s = u_s / u_c for dx = 1."""
    D = (12 * g * g + 12 * g * (ts - 1) + (2 * ts - 1) * (4 * l * tq - 1 - 4 * tq)
         - l * (11 * (2 * ts - 1) + 12 * g * ts))
    return (2 * (1 + l) * (1 - r) / r * ts / h
            - (1.0 / (3 * r)) * ((1 + l) * (1 + 4 * tq - 2 * ts + 12 * g * ts - 8 * ts * tq) + r * D) / h ** 2)


def slip_numerislip(r, l, g, ts, tq, kn):
    """Eq. (NumeriSlip): the same slip written with Kn through Eq. (tKnrela)."""
    K = ((2 * ts - 1) * (1 + r + l + 11 * l * r) + 12 * g * (r + ts * (l * r - l - r - 1)) - 12 * r * g * g
         - 4 * tq * (2 * ts - 1) * (l * r - l - r - 1))
    return (4 * (1 - r) * (1 + l) * ts / (r * (2 * ts - 1)) * SQ6PI * kn
            + 8 / math.pi * K / (r * (2 * ts - 1) ** 2) * kn * kn)


def slip_physical(L1, L2, kn):
    """Eq. (PhyscPoiSlip): U_s = 4 L1 Kn + 8 L2 Kn^2."""
    return 4 * L1 * kn + 8 * L2 * kn * kn


def r_slicoeffrtsr(l, ts, L1):
    """Eq. (SliCoeffrtsr)."""
    return SQ6PI * ts * (1 + l) / (L1 * (2 * ts - 1) + SQ6PI * ts * (1 + l))


def tau_q_slicoeffrtstq(g, l, ts, L1, L2):
    """Eq. (SliCoeffrtstq)."""
    num = (L1 * (2 * ts - 1) * (2 * ts * (6 * g - 1) + 1)
           + SQ6PI * ts * (L2 * math.pi * (2 * ts - 1) ** 2 + 12 * g * g + 2 * (2 * ts - 1) * (6 * g - 6 * l - 1)))
    return num / (4 * (2 * ts - 1) * (2 * SQ6PI * ts + L1 * (2 * ts - 1)))


def tau_q_halfway(ts, L1, L2):
    """Eq. (SliCoeffHata): halfway DBB (gamma = 1/2, l = 0)."""
    num = L1 * (2 * ts - 1) * (4 * ts + 1) + SQ6PI * ts * (L2 * math.pi * (2 * ts - 1) ** 2 + 4 * (2 * ts - 1) + 3)
    return num / (4 * (2 * ts - 1) * (2 * SQ6PI * ts + L1 * (2 * ts - 1)))


def l_eqexlva(g, ts, L1, E):
    """Eq. (Eqexlva)."""
    return (SQ6PI * g * g + g * (2 * ts - 1) * (L1 + SQ6PI)) / (SQ6PI * (2 * ts - 1)) + E


def e_upper(ts, L1, L2):
    """Eq. (EqECond), right-hand side."""
    return (math.pi * ts * L2 - 3 * math.sqrt(math.pi / 6) * L1) * (2 * ts - 1) / (12 * ts) - 0.5


def poiseuille_profile(y, h, L1, L2, kn):
    """Eq. (numvelo): U(y) = 4 (y/H)(1 - y/H) + 4 L1 Kn + 8 L2 Kn^2."""
    return 4 * y / h * (1 - y / h) + slip_physical(L1, L2, kn)


def couette_utheta(rr, R1, R2, w1, w2, lam, s1=1.0, s2=1.0):
    """Eqs. (EqAnaMicro)-(EqAnaPraMicro): tangential velocity between rotating cylinders."""
    Mc = (1 / R2 ** 2) * (1 - (2 - s2) / s2 * 2 * lam / R2)
    Nc = (1 / R1 ** 2) * (1 + (2 - s1) / s1 * 2 * lam / R1)
    return (Mc * w1 - Nc * w2) / (Mc - Nc) * rr + (w1 - w2) / (Nc - Mc) / rr
