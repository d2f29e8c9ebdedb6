"""ImEx additive Runge-Kutta stepping, embedded error, WRMS norm, step control (FP64 oracle).

Follows Methods, "Time integration": the stage equation and update of the
ImEx-ARK pair (Eq. ARK_method with Eq. ARK_stage), the embedded solution
(Eq. ARK_embedding), the local truncation error as the difference of the two,
the WRMS norm (Eq. wrms_norm) with weights (Eq. wrms_weights), and the
accept-if-norm-at-most-one rule.  Only the stiff linear terms are implicit,
so each implicit stage solve is a division by ``1 - dt A^I_ii L(k)`` per mode.

Tables: first-order IMEX Euler (2-stage ARK form); the second-order
three-stage ARK2 of Giraldo, Kelly & Constantinescu (2013, SIAM J. Sci.
Comput. 35), whose entries lie in Q(sqrt 2) and are kept exactly as
a + b sqrt 2; ARK3(2)4L[2]SA and ARK4(3)6L[2]SA of Kennedy & Carpenter (2003,
Appl. Numer. Math. 44), the third- and fourth-order methods the paper's
order study cites; their coefficients are the published rationals.

Readings (where the paper leaves a choice): the WRMS vector is the reciprocal-space state
scaled to unit norm (Parseval), modes weighted by their half-spectrum
multiplicity (default), or the real-space state itself (``norm_space = 1``:
the norm and weights of Eqs. wrms_norm / wrms_weights applied point by point
to the four real fields); the step-size controller, which the paper leaves to
the library, is the elementary I-controller
``dt * min(5, max(0.2, 0.9 err^(-1/(q+1))))`` with embedding order q, a factor
0.25 after a non-finite result, and no growth (factor at most 1) for the step
proposed after an accepted attempt that directly follows a rejected one
(Hairer, Norsett & Wanner, Solving ODEs I, section II.4: facmax = 1 right after
a rejection).

Pinned by tests/test_oracle_ark.py: order conditions in exact rational
arithmetic, row sums, the closed-form stability function on a scalar linear
test problem, IMEX Euler against its direct formula, WRMS on hand vectors
(both norm spaces, the k-space norm with a relative tolerance on a hand-worked
single-mode case), observed convergence orders, and the controller's
reject-accept sequence in the time loop.
"""
from __future__ import annotations

from fractions import Fraction as Fr

import numpy as np

from . import spectral as sp


class Table:
    """Paired Butcher tables (A^E, A^I, b, b~, c) with exact rational entries."""

    def __init__(self, name, AE, AI, b, bt, c, order, emb_order, bI=None):
        self.name = name
        self.s = len(c)
        self.AE_q, self.AI_q = AE, AI
        self.b_q, self.bt_q, self.c_q = b, bt, c
        self.bI_q = b if bI is None else bI
        self.AE = np.array([[float(x) for x in row] for row in AE])
        self.AI = np.array([[float(x) for x in row] for row in AI])
        self.b = np.array([float(x) for x in b])          # explicit weights b^E
        self.bI = np.array([float(x) for x in self.bI_q])  # implicit weights b^I
        self.bt = None if bt is None else np.array([float(x) for x in bt])
        self.c = np.array([float(x) for x in c])
        self.order = order
        self.emb_order = emb_order

    def explicit_needed(self, i):
        """Whether f^E at stage i is used by any later stage, the update or the embedding."""
        used = self.b[i] != 0.0 or (self.bt is not None and self.bt[i] != 0.0)
        return used or bool(np.any(self.AE[i + 1:, i] != 0.0))


def _q(s):
    return Fr(s)


class QS2:
    """Exact element a + b sqrt(2) of Q(sqrt 2), a and b rational."""

    def __init__(self, a, b=0):
        self.a, self.b = Fr(a), Fr(b)

    @staticmethod
    def _c(x):
        return x if isinstance(x, QS2) else QS2(x)

    def __add__(self, o):
        o = QS2._c(o)
        return QS2(self.a + o.a, self.b + o.b)

    __radd__ = __add__

    def __neg__(self):
        return QS2(-self.a, -self.b)

    def __sub__(self, o):
        return self + (-QS2._c(o))

    def __rsub__(self, o):
        return QS2._c(o) - self

    def __mul__(self, o):
        o = QS2._c(o)
        return QS2(self.a * o.a + 2 * self.b * o.b, self.a * o.b + self.b * o.a)

    __rmul__ = __mul__

    def __pow__(self, k):
        out = QS2(1)
        for _ in range(int(k)):
            out = out * self
        return out

    def __eq__(self, o):
        o = QS2._c(o)
        return self.a == o.a and self.b == o.b

    def __ne__(self, o):
        return not self == o

    def __hash__(self):
        return hash((self.a, self.b))

    def __float__(self):
        # a + b sqrt 2 in long double-free form: the two rationals in binary64 (the
        # product's rounding error is below 2^-52 of the magnitude)
        return float(self.a) + float(self.b) * 2.0 ** 0.5

    def __repr__(self):
        return "QS2(%s, %s)" % (self.a, self.b)


def imex_euler():
    """First-order IMEX Euler as a 2-stage ARK pair (explicit first stage, implicit second)."""
    z, o = Fr(0), Fr(1)
    return Table("imex_euler",
                 AE=[[z, z], [o, z]], AI=[[z, z], [z, o]],
                 b=[o, z], bI=[z, o], bt=None, c=[z, o], order=1, emb_order=None)


def ark436l2sa():
    """ARK4(3)6L[2]SA, Kennedy & Carpenter 2003: 6 stages, ESDIRK implicit part, gamma = 1/4."""
    q = _q
    AE = [[0] * 6 for _ in range(6)]
    AE[1][0] = q("1/2")
    AE[2][0], AE[2][1] = q("13861/62500"), q("6889/62500")
    AE[3][0], AE[3][1], AE[3][2] = (q("-116923316275/2393684061468"),
                                    q("-2731218467317/15368042101831"),
                                    q("9408046702089/11113171139209"))
    AE[4][0], AE[4][1], AE[4][2], AE[4][3] = (q("-451086348788/2902428689909"),
                                              q("-2682348792572/7519795681897"),
                                              q("12662868775082/11960479115383"),
                                              q("3355817975965/11060851509271"))
    AE[5][0], AE[5][1], AE[5][2], AE[5][3], AE[5][4] = (q("647845179188/3216320057751"),
                                                        q("73281519250/8382639484533"),
                                                        q("552539513391/3454668386233"),
                                                        q("3354512671639/8306763924573"),
                                                        q("4040/17871"))
    b = [q("82889/524892"), q(0), q("15625/83664"), q("69875/102672"),
         q("-2260/8211"), q("1/4")]
    bt = [q("4586570599/29645900160"), q(0), q("178811875/945068544"),
          q("814220225/1159782912"), q("-3700637/11593932"), q("61727/225920")]
    g = q("1/4")
    AI = [[q(0)] * 6 for _ in range(6)]
    AI[1][0], AI[1][1] = g, g
    AI[2][0], AI[2][1], AI[2][2] = q("8611/62500"), q("-1743/31250"), g
    AI[3][0], AI[3][1], AI[3][2], AI[3][3] = (q("5012029/34652500"), q("-654441/2922500"),
                                              q("174375/388108"), g)
    AI[4][0], AI[4][1], AI[4][2], AI[4][3], AI[4][4] = (q("15267082809/155376265600"),
                                                        q("-71443401/120774400"),
                                                        q("730878875/902184768"),
                                                        q("2285395/8070912"), g)
    AI[5] = list(b)
    AE = [[q(x) if not isinstance(x, Fr) else x for x in row] for row in AE]
    c = [q(0), q("1/2"), q("83/250"), q("31/50"), q("17/20"), q(1)]
    return Table("ark436l2sa", AE=AE, AI=AI, b=b, bt=bt, c=c, order=4, emb_order=3)


def ark2():
    """ARK2 of Giraldo, Kelly & Constantinescu (2013): 3 stages, second order,
    ESDIRK implicit part with gamma = 1 - 1/sqrt 2, stiffly accurate, explicit
    weight alpha = (3 + 2 sqrt 2)/6 in the last row, embedded first-order
    weights ((4 - sqrt 2)/8, (4 - sqrt 2)/8, 1/(2 sqrt 2))."""
    z = QS2(0)
    g = QS2(1, Fr(-1, 2))            # 1 - sqrt(2)/2
    d = QS2(0, Fr(1, 4))             # sqrt(2)/4 = 1/(2 sqrt 2)
    al = QS2(Fr(1, 2), Fr(1, 3))     # (3 + 2 sqrt 2)/6
    c = [z, 2 * g, QS2(1)]
    AE = [[z, z, z], [2 * g, z, z], [1 - al, al, z]]
    AI = [[z, z, z], [g, g, z], [d, d, g]]
    b = [d, d, g]
    bt = [QS2(Fr(1, 2), Fr(-1, 8)), QS2(Fr(1, 2), Fr(-1, 8)), QS2(0, Fr(1, 4))]
    return Table("ark2", AE=AE, AI=AI, b=b, bt=bt, c=c, order=2, emb_order=1)


def ark324l2sa():
    """ARK3(2)4L[2]SA, Kennedy & Carpenter 2003: 4 stages, ESDIRK implicit part,
    stiffly accurate, embedded second-order weights."""
    q = _q
    g = q("1767732205903/4055673282236")
    z = q(0)
    AE = [[z] * 4 for _ in range(4)]
    AE[1][0] = q("1767732205903/2027836641118")
    AE[2][0], AE[2][1] = q("5535828885825/10492691773637"), q("788022342437/10882634858940")
    AE[3][0], AE[3][1], AE[3][2] = (q("6485989280629/16251701735622"), q("-4246266847089/9704473918619"),
                                    q("10755448449292/10357097424841"))
    b = [q("1471266399579/7840856788654"), q("-4482444167858/7529755066697"),
         q("11266239266428/11593286722821"), q("1767732205903/4055673282236")]
    bt = [q("2756255671327/12835298489170"), q("-10771552573575/22201958757719"),
          q("9247589265047/10645013368117"), q("2193209047091/5459859503100")]
    AI = [[z] * 4 for _ in range(4)]
    AI[1][0], AI[1][1] = q("1767732205903/4055673282236"), g
    AI[2][0], AI[2][1], AI[2][2] = q("2746238789719/10658868560708"), q("-640167445237/6845629431997"), g
    AI[3] = list(b)
    c = [z, q("1767732205903/2027836641118"), q("3/5"), q(1)]
    return Table("ark324l2sa", AE=AE, AI=AI, b=b, bt=bt, c=c, order=3, emb_order=2)


TABLES = {"imex_euler": imex_euler, "ark2": ark2, "ark324l": ark324l2sa, "ark436l": ark436l2sa}


def ark_step(y, dt, table, f_explicit, Lsym):
    """One ImEx-ARK step for ``y' = L y + f_E(y)`` with diagonal ``L``.

    Stage i: ``r_i = y + dt sum_{j<i} (A^E_ij F^E_j + A^I_ij F^I_j)``, then the
    implicit stage solve ``z_i = r_i / (1 - dt A^I_ii L)``, ``F^I_i = L z_i``
    and ``F^E_i = f_E(z_i)`` when later used.  Returns ``(y_new, lte, n_explicit)``
    with ``y_new = y + dt sum_i (b^I_i F^I_i + b^E_i F^E_i)`` and
    ``lte = dt sum_i (b_i - b~_i)(F^I_i + F^E_i)`` (None without embedding;
    the embedded pairs used here share b^I = b^E and b~^I = b~^E).
    """
    s = table.s
    FI = [None] * s
    FE = [None] * s
    n_exp = 0
    for i in range(s):
        r = y.copy()
        for j in range(i):
            if table.AE[i, j] != 0.0:
                r = r + dt * table.AE[i, j] * FE[j]
            if table.AI[i, j] != 0.0:
                r = r + dt * table.AI[i, j] * FI[j]
        z = r / (1.0 - dt * table.AI[i, i] * Lsym) if table.AI[i, i] != 0.0 else r
        FI[i] = Lsym * z
        if table.explicit_needed(i):
            FE[i] = f_explicit(z)
            n_exp += 1
        else:
            FE[i] = np.zeros_like(z)
    incr = np.zeros_like(y)
    for i in range(s):
        if table.bI[i] != 0.0:
            incr = incr + table.bI[i] * FI[i]
        if table.b[i] != 0.0:
            incr = incr + table.b[i] * FE[i]
    y_new = y + dt * incr
    lte = None
    if table.bt is not None:
        d = np.zeros_like(y)
        for i in range(s):
            coef = table.b[i] - table.bt[i]
            if coef != 0.0:
                d = d + coef * (FI[i] + FE[i])
        lte = dt * d
    return y_new, lte, n_exp


def imex_euler_direct(y, dt, f_explicit, Lsym):
    """IMEX Euler written directly: ``y_new = (y + dt f_E(y)) / (1 - dt L)``."""
    return (y + dt * f_explicit(y)) / (1.0 - dt * Lsym)


def wrms(v, w):
    """Weighted root-mean-square norm ``sqrt(mean((v w)^2))`` (Eq. wrms_norm)."""
    v = np.asarray(v)
    return float(np.sqrt(np.mean((np.abs(v) * w) ** 2)))


def wrms_weights(y_prev, rtol, atol):
    """``w_i = 1 / (rtol |y_prev,i| + atol)`` (Eq. wrms_weights)."""
    return 1.0 / (rtol * np.abs(y_prev) + atol)


def wrms_kspace(lte_hat, y_prev_hat, rtol, atol, mult, n3):
    """WRMS of a half-spectrum error over all fields, as a real-space-equivalent RMS.

    Coefficients are scaled by ``1/sqrt(N^3)`` (unitary DFT) so that uniform
    weights give the real-space RMS by Parseval; each half-spectrum mode counts
    ``mult`` times and the vector length is ``fields * N^3``.
    """
    s = 1.0 / np.sqrt(n3)
    e = np.abs(lte_hat) * s
    w = 1.0 / (rtol * np.abs(y_prev_hat) * s + atol)
    nf = lte_hat.shape[0]
    tot = float(np.sum(mult * (e * w) ** 2))
    return float(np.sqrt(tot / (nf * n3)))


def wrms_real(lte_hat, y_prev_hat, rtol, atol, shape):
    """WRMS of the error in real space (``norm_space = 1``): Eq. wrms_norm with the
    weights of Eq. wrms_weights taken point by point over every real field, vector
    length ``fields * N^3``."""
    e = sp.irfft3(lte_hat, shape)
    yp = sp.irfft3(y_prev_hat, shape)
    return wrms(e, wrms_weights(yp, rtol, atol))


def controller(dt, err, q, after_reject=False):
    """Elementary I-controller: next step size from the WRMS error estimate.

    ``after_reject``: this attempt was accepted and the one before it was
    rejected; the proposal then does not grow (factor capped at 1).
    """
    if not np.isfinite(err):
        return 0.25 * dt
    if err == 0.0:
        fac = 5.0
    else:
        fac = min(5.0, max(0.2, 0.9 * err ** (-1.0 / (q + 1))))
    if after_reject:
        fac = min(1.0, fac)
    return dt * fac


class Integrator:
    """Fixed or adaptive time loop over :func:`ark_step` (host-side control, FP64)."""

    def __init__(self, model, table="ark436l", adaptive=False, dt0=1e-2, rtol=1e-6,
                 atol=1e-9, dt_min=0.0, dt_max=np.inf, max_rejects=10, norm_space=0):
        self.model = model
        self.table = TABLES[table]() if isinstance(table, str) else table
        self.adaptive = bool(adaptive)
        if self.adaptive and self.table.bt is None:
            raise ValueError("adaptive stepping needs an embedded method")
        self.dt = float(dt0)
        self.rtol, self.atol = float(rtol), float(atol)
        self.dt_min, self.dt_max = float(dt_min), float(dt_max)
        self.max_rejects = int(max_rejects)
        self.norm_space = int(norm_space)
        self.Lsym = model.implicit_symbol()
        self.prev_rejected = False
        # log: one (t, dt, err, accepted, dt_next) tuple per attempt
        self.stats = dict(steps=0, attempts=0, rejects=0, n_rhs=0, dts=[], errs=[], log=[])

    def attempt(self, y, dt):
        y_new, lte, n_exp = ark_step(y, dt, self.table, self.model.f_explicit, self.Lsym)
        self.stats["n_rhs"] += n_exp
        self.stats["attempts"] += 1
        err = 0.0
        if lte is not None:
            if self.norm_space == 1:
                err = wrms_real(lte, y, self.rtol, self.atol, self.model.shape)
            else:
                err = wrms_kspace(lte, y, self.rtol, self.atol, self.model.mult, self.model.N3)
        finite = bool(np.all(np.isfinite(y_new))) and np.isfinite(err)
        return y_new, (err if finite else np.inf)

    def advance(self, y, t, t_final, dt_sequence=None, max_steps=None):
        """Integrate from t to t_final; returns (y, t).  Replays ``dt_sequence`` if given;
        stops after ``max_steps`` accepted steps if given."""
        rejects = 0
        accepted = 0
        seq = list(dt_sequence) if dt_sequence is not None else None
        while (t < t_final * (1.0 - 1e-15) and (seq is None or seq)
               and (max_steps is None or accepted < max_steps)):
            dt = seq.pop(0) if seq is not None else min(self.dt, self.dt_max)
            dt = min(dt, t_final - t)
            y_new, err = self.attempt(y, dt)
            ok = np.isfinite(err) and (not self.adaptive or err <= 1.0 or seq is not None)
            if self.adaptive:
                cap = ok and self.prev_rejected
                self.dt = controller(dt, err, self.table.emb_order, after_reject=cap)
                self.dt = max(self.dt, self.dt_min)
                self.prev_rejected = not ok
            elif not np.isfinite(err):
                raise FloatingPointError("non-finite state in fixed-step run")
            self.stats["log"].append((t, dt, err, bool(ok), self.dt))
            if ok:
                y, t = y_new, t + dt
                accepted += 1
                self.stats["steps"] += 1
                self.stats["dts"].append(dt)
                self.stats["errs"].append(err)
                rejects = 0
            else:
                self.stats["rejects"] += 1
                rejects += 1
                if rejects >= self.max_rejects:
                    raise RuntimeError("step failed after %d consecutive rejections" % rejects)
        return y, t
