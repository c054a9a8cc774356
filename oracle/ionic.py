"""Ionic models for the oracle, vectorised over nodes.  FP64 numpy.
Test infrastructure only.

Every model exposes, per node:
  * ``gates(V)`` -> (Lambda_E, z_inf) with Lambda_E = -(alpha + beta) and
    z_inf = alpha/(alpha + beta)  (gate equation of the monodomain model,
    rewritten in exponential form; the printed formula for z_inf carries a
    spurious minus sign, the reading used here is the one consistent with
    the gate ODE alpha(1 - z) - beta z);
  * ``i_ion(V, zE, zS)`` -> ionic current per unit membrane capacitance
    (mV/ms), so that the paper's I_ion equals Cm * i_ion;
  * ``g_S(V, zE, zS)`` -> time derivatives of the non-gate variables;
  * ``rest()`` -> the uniform initial state (V, z_E, z_S).

HH is the classical 1952 Hodgkin-Huxley squid-axon model (modern sign
convention, rest near -65 mV).  CRN_SURR and TTP_SURR are project-written
surrogates: they are NOT the Courtemanche-Ramirez-Nattel or ten
Tusscher-Panfilov models, whose definitions are not available here.  They
reproduce those models' sizes (20 and 18 ionic variables, split 15+5 and
12+6 between gates and other variables) and their stiffness (largest gate
rate about 130/ms and 1000/ms), with an HH excitable core whose
conductances are scaled to cardiac magnitudes (one tenth of the squid-axon
values), extra gated currents and concentration-like slow variables.  Their formulas are
definitions of this project; their single-cell trajectories are pinned
against a library ODE integrator in the tests, multi-node trajectories are
parity unpinned.
"""
import numpy as np

RTF = 25.69          # RT/F in mV
NA_O, K_O, CA_O = 140.0, 5.4, 1.8
NA_I0, K_I0, CA_I0 = 20.0, 108.0, 1e-4
SERIES_EPS = 1e-7    # below this |x|, x/expm1(x) is replaced by its series


def _x_over_expm1(x):
    """x/(e^x - 1) with its removable singularity at x = 0 (1 - x/2 there)."""
    small = np.abs(x) < SERIES_EPS
    xs = np.where(small, 1.0, x)
    return np.where(small, 1.0 - 0.5 * x, xs / np.expm1(xs))


def hh_core_rates(V, km):
    """(alpha, beta) for the HH gates m, h, n; the m rates are scaled by km."""
    am = _x_over_expm1(-(V + 40.0) / 10.0)
    bm = 4.0 * np.exp(-(V + 65.0) / 18.0)
    ah = 0.07 * np.exp(-(V + 65.0) / 20.0)
    bh = 1.0 / (1.0 + np.exp(-(V + 35.0) / 10.0))
    an = 0.1 * _x_over_expm1(-(V + 55.0) / 10.0)
    bn = 0.125 * np.exp(-(V + 65.0) / 80.0)
    return [(km * am, km * bm), (ah, bh), (an, bn)]


def sigmoid_rates(V, A, Va, sa, Vb, sb):
    """alpha = A/(1 + exp(-(V - Va)/sa)), beta = A/(1 + exp((V - Vb)/sb))."""
    alpha = A / (1.0 + np.exp(-(V - Va) / sa))
    beta = A / (1.0 + np.exp((V - Vb) / sb))
    return alpha, beta


def _lambda_inf(rates):
    lam = np.stack([-(a + b) for a, b in rates])
    zinf = np.stack([a / (a + b) for a, b in rates])
    return lam, zinf


class HH:
    name = "HH"
    n_gates = 3
    n_slow = 0
    V_REST = -65.0

    def rates(self, V):
        return hh_core_rates(V, 1.0)

    def gates(self, V):
        return _lambda_inf(self.rates(V))

    def i_ion(self, V, zE, zS):
        m, h, n = zE[0], zE[1], zE[2]
        return (120.0 * m ** 3 * h * (V - 50.0) + 36.0 * n ** 4 * (V + 77.0)
                + 0.3 * (V + 54.387))

    def g_S(self, V, zE, zS):
        return np.zeros((0,) + np.shape(V))

    def rest(self):
        V = np.array([self.V_REST])
        _, zinf = self.gates(V)
        return np.concatenate([V, zinf[:, 0]])


class LinearTest:
    """I_ion = Cm * a * V and one decoupled gate with constant Lambda = lam_E
    and z_inf = 0 (linear test problem of the stability analysis)."""
    name = "LINEAR"
    n_gates = 1
    n_slow = 0

    def __init__(self, a=0.0, lam_E=0.0):
        self.a = float(a)
        self.lam_E = float(lam_E)

    def gates(self, V):
        V = np.asarray(V, dtype=np.float64)
        return np.full((1,) + V.shape, self.lam_E), np.zeros((1,) + V.shape)

    def i_ion(self, V, zE, zS):
        return self.a * V

    def g_S(self, V, zE, zS):
        return np.zeros((0,) + np.shape(V))

    def rest(self):
        return np.zeros(2)


# Surrogate gate tables: rows (A, Va, sa, Vb, sb) for sigmoid_rates.
CRN_SURR_GATES = (
    (2.0, -20.0, 10.0, -12.0, 13.0),
    (0.06, -50.0, -8.0, -58.0, -10.4),
    (0.4, -10.0, 12.0, -2.0, 15.6),
    (0.004, -40.0, -10.0, -48.0, -13.0),
    (1.0, -15.0, 6.0, -7.0, 7.8),
    (0.02, -30.0, -7.0, -38.0, -9.1),
    (0.02, -15.0, 8.0, -7.0, 10.4),
    (1.0, -40.0, -20.0, -48.0, -26.0),
    (0.006, 10.0, 15.0, 18.0, 19.5),
    (0.008, 5.0, 13.0, 13.0, 16.9),
    (0.2, -30.0, -10.0, -38.0, -13.0),
    (0.04, 0.0, 10.0, 8.0, 13.0),
)

TTP_SURR_GATES = (
    (3.0, -25.0, 9.0, -17.0, 11.7),
    (0.08, -45.0, -7.0, -53.0, -9.1),
    (0.03, -20.0, 9.0, -12.0, 11.7),
    (1.5, -45.0, -18.0, -53.0, -23.4),
    (0.01, 5.0, 14.0, 13.0, 18.2),
    (1.5, -12.0, 6.0, -4.0, 7.8),
    (0.03, -28.0, -7.0, -36.0, -9.1),
    (0.3, -35.0, -6.0, -43.0, -7.8),
    (0.5, -10.0, 8.0, -2.0, 10.4),
)


class _Surrogate:
    KM = 1.0
    TABLE = ()
    SLOW_REST = ()
    V_REST = -65.0

    @property
    def n_gates(self):
        return 3 + len(self.TABLE)

    @property
    def n_slow(self):
        return len(self.SLOW_REST)

    def rates(self, V):
        r = hh_core_rates(V, self.KM)
        for row in self.TABLE:
            r.append(sigmoid_rates(V, *row))
        return r

    def gates(self, V):
        return _lambda_inf(self.rates(V))

    def rest(self):
        V = np.array([self.V_REST])
        _, zinf = self.gates(V)
        return np.concatenate([V, zinf[:, 0], np.asarray(self.SLOW_REST, dtype=np.float64)])


class CRNSurrogate(_Surrogate):
    """CRN-shaped surrogate: V + 15 gates (m, h, n, g3..g14) + 5 slow
    variables (Na_i, K_i, Ca_i, Ca_up, Ca_rel)."""
    name = "CRN_SURR"
    KM = 15.0
    TABLE = CRN_SURR_GATES
    SLOW_REST = (NA_I0, K_I0, CA_I0, 1.0, 1.0)
    J_LEAK = 0.005 * CA_I0 / (CA_I0 + 0.001)

    def _currents(self, V, zE, zS):
        m, h, n = zE[0], zE[1], zE[2]
        g = zE
        Na, K, Ca = zS[0], zS[1], zS[2]
        ENa = RTF * np.log(NA_O / Na)
        EK = RTF * np.log(K_O / K)
        ECa = 0.5 * RTF * np.log(CA_O / Ca)
        iNa = 12.0 * m ** 3 * h * (V - ENa)
        iK = 3.6 * n ** 4 * (V - EK)
        iL = 0.03 * (V + 54.387)
        ito = 0.04 * g[3] ** 3 * g[4] * (V - EK)
        ikur = 0.02 * g[5] ** 3 * g[6] * (V - EK)
        ical = 0.03 * g[7] * g[8] * (V - ECa)
        ikr = 0.02 * g[9] * g[10] * (V - EK)
        iks = 0.01 * g[11] * g[12] * (V - EK)
        ik1 = 0.005 * (V - EK) / (1.0 + np.exp(0.07 * (V + 80.0)))
        return iNa, iK, iL, ito, ikur, ical, ikr, iks, ik1

    def i_ion(self, V, zE, zS):
        iNa, iK, iL, ito, ikur, ical, ikr, iks, ik1 = self._currents(V, zE, zS)
        return iNa + iK + iL + ito + ikur + ical + ikr + iks + ik1

    def g_S(self, V, zE, zS):
        iNa, iK, iL, ito, ikur, ical, ikr, iks, ik1 = self._currents(V, zE, zS)
        g = zE
        Na, K, Ca, Cup, Crel = zS[0], zS[1], zS[2], zS[3], zS[4]
        jrel = 0.5 * g[13] ** 2 * g[14] * (Crel - Ca)
        jup = 0.005 * Ca / (Ca + 0.001)
        jtr = (Cup - Crel) / 50.0
        dNa = -1e-4 * iNa + (NA_I0 - Na) / 500.0
        dK = -1e-4 * (iK + ito + ikur + ikr + iks + ik1) + (K_I0 - K) / 500.0
        dCa = -2e-6 * ical + 0.02 * jrel - jup + self.J_LEAK + (CA_I0 - Ca) / 100.0
        dCup = 0.05 * jup - 0.05 * jtr
        dCrel = 0.05 * jtr - 0.001 * jrel
        return np.stack([dNa, dK, dCa, dCup, dCrel])


class TTPSurrogate(_Surrogate):
    """TTP-shaped surrogate: V + 12 gates (m, h, n, g3..g11) + 6 slow
    variables (Na_i, K_i, Ca_i, Ca_sr, Ca_ss, R)."""
    name = "TTP_SURR"
    KM = 110.0
    TABLE = TTP_SURR_GATES
    SLOW_REST = (NA_I0, K_I0, CA_I0, 1.0, 1e-4, 0.98)
    J_LEAK = 0.004 * CA_I0 / (CA_I0 + 0.00025)

    def _currents(self, V, zE, zS):
        m, h, n = zE[0], zE[1], zE[2]
        g = zE
        Na, K, Css = zS[0], zS[1], zS[4]
        ENa = RTF * np.log(NA_O / Na)
        EK = RTF * np.log(K_O / K)
        ECa = 0.5 * RTF * np.log(CA_O / Css)
        iNa = 12.0 * m ** 3 * h * (V - ENa)
        iK = 3.6 * n ** 4 * (V - EK)
        iL = 0.03 * (V + 54.387)
        ito = 0.03 * g[3] ** 3 * g[4] * (V - EK)
        ikr = 0.015 * g[5] * g[6] * (V - EK)
        iks = 0.01 * g[7] ** 2 * (V - EK)
        ical = 0.025 * g[8] * g[9] * g[10] * (V - ECa)
        ik1 = 0.005 * (V - EK) / (1.0 + np.exp(0.07 * (V + 80.0)))
        return iNa, iK, iL, ito, ikr, iks, ical, ik1

    def i_ion(self, V, zE, zS):
        iNa, iK, iL, ito, ikr, iks, ical, ik1 = self._currents(V, zE, zS)
        return iNa + iK + iL + ito + ikr + iks + ical + ik1

    def g_S(self, V, zE, zS):
        iNa, iK, iL, ito, ikr, iks, ical, ik1 = self._currents(V, zE, zS)
        g = zE
        Na, K, Ca, Csr, Css, R = zS[0], zS[1], zS[2], zS[3], zS[4], zS[5]
        jrel = 0.4 * g[11] * R * (Csr - Css)
        jup = 0.004 * Ca / (Ca + 0.00025)
        jxfer = (Css - Ca) / 2.0
        dNa = -1e-4 * iNa + (NA_I0 - Na) / 500.0
        dK = -1e-4 * (iK + ito + ikr + iks + ik1) + (K_I0 - K) / 500.0
        dCa = 0.1 * jxfer - jup + self.J_LEAK + (CA_I0 - Ca) / 100.0
        dCsr = 0.02 * (jup - self.J_LEAK) - 0.002 * jrel
        dCss = -2e-6 * ical + 0.01 * jrel - jxfer
        dR = (0.98 - R) / 200.0 - 5.0 * (Css - 1e-4) * R
        return np.stack([dNa, dK, dCa, dCsr, dCss, dR])


def make_model(name, **kw):
    if name == "HH":
        return HH()
    if name == "LINEAR":
        return LinearTest(**kw)
    if name == "CRN_SURR":
        return CRNSurrogate()
    if name == "TTP_SURR":
        return TTPSurrogate()
    raise ValueError(name)
