"""FP64 reference of the unrolled EWAInit-BP and Momentum-BP soft loss and its gradient.

TEST INFRASTRUCTURE: only the tests and the benchmark's reference leg use it;
it shares nothing with the GPU library.

The forward is EWAInit-BP (section III-B, eq. EWAInit and Algorithm 2) or
Momentum-BP (section III-A1, eqs. mombp1-3) over GF(4) in the flooding schedule
(check and qubit rules of section II-B1) run for a fixed number T of iterations
with no early stop, with learnable per-iteration parameters and priors Pi^{(0)}:
EWAInit a discount alpha_t per iteration (alpha_1 unused: Pi^{(1)} = Pi^{(0)});
Momentum a step alpha_t and a decay gamma_t per iteration (params [T, 2]):
g^{(t)} = gamma_t g^{(t-1)} + (1 - gamma_t)(Q^{(t-1)} - Pi^{(0)} - M^{(t)}),
Q^{(t)} = Q^{(t-1)} - alpha_t g^{(t)}, g^{(0)} = 0, Q^{(0)} = Pi^{(0)}.
The loss is the mean over shots and qubits of the negative log GF(4) marginal
of the sampled error at iteration T, with P_v(I) prop. to 1 and P_v(W) prop.
to exp(-Q_W):  ln(1 + sum_W exp(-Q_W)) + Q_{e_v}  (Q_I = 0).
The gradient with respect to the per-iteration parameters and Pi^{(0)} is torch
autograd in float64 on the CPU.  Every step is written as the formula it implements, with
whole-batch tensor operations and no reordering beyond plain sums.
"""
from __future__ import annotations

import numpy as np
import torch

F64 = torch.float64
# Q index (X, Y, Z order) of a Pauli code (bit0 x, bit1 z): X=1 -> 0, Y=3 -> 1, Z=2 -> 2
Q_INDEX = {1: 0, 3: 1, 2: 2}
# for an edge label H: the index of H and of the two Paulis that anticommute with H
LABEL_H = {1: 0, 2: 2, 3: 1}
LABEL_PAIR = {1: (1, 2), 2: (0, 1), 3: (0, 2)}


def _edges(hx, hz):
    """Nonzeros of H in row-major order: check, qubit, label (X=1, Z=2, Y=3)."""
    lab = (np.asarray(hx, np.uint8) & 1) | ((np.asarray(hz, np.uint8) & 1) << 1)
    c, v = np.nonzero(lab)
    return c, v, lab[c, v]


def phi(x):
    """phi(x) = -ln tanh(x / 2) = ln(1 + 2 / (e^x - 1)), x >= 0 (eq. h_update in magnitude form)."""
    return torch.log1p(2.0 / torch.expm1(x))


class Tanner:
    """Index tables of one check matrix for the batched reference."""

    def __init__(self, hx, hz):
        hx = np.asarray(hx, np.uint8)
        self.m, self.n = hx.shape
        c, v, lab = _edges(hx, hz)
        E = len(c)
        self.E = E
        self.check = torch.as_tensor(c, dtype=torch.long)
        self.qubit = torch.as_tensor(v, dtype=torch.long)
        self.label = lab
        # the other edges of each edge's check, padded with E (a column of phi = 0, sign = +1)
        others = np.full((E, 3), E, np.int64)
        for e in range(E):
            o = [f for f in np.nonzero(c == c[e])[0] if f != e]
            if len(o) > 3:
                raise ValueError("check degree above 4")
            others[e, :len(o)] = o
        self.others = torch.as_tensor(others)
        # (qubit, X/Y/Z index) of H and of its anticommuting pair, per edge
        self.h_idx = torch.as_tensor([3 * v[e] + LABEL_H[int(lab[e])] for e in range(E)])
        self.a_idx = torch.as_tensor([3 * v[e] + LABEL_PAIR[int(lab[e])][0] for e in range(E)])
        self.b_idx = torch.as_tensor([3 * v[e] + LABEL_PAIR[int(lab[e])][1] for e in range(E)])
        # M_{v,W} = sum of m_{c->v} over edges of v whose label anticommutes with W
        A = torch.zeros(E, 3 * self.n, dtype=F64)
        for e in range(E):
            A[e, self.a_idx[e]] = 1.0
            A[e, self.b_idx[e]] = 1.0
        self.A = A


def lam(tg: Tanner, Q):
    """lambda_{H}(Q_v) = ln(1 + e^{-Q_H}) - ln(e^{-Q_a} + e^{-Q_b}) per edge; Q is [shots, 3n]."""
    zero = torch.zeros((), dtype=F64)
    return (torch.logaddexp(zero, -Q[:, tg.h_idx])
            - torch.logaddexp(-Q[:, tg.a_idx], -Q[:, tg.b_idx]))


def forward(tg: Tanner, alpha, prior, synd, err, T: int, clamp: float = 30.0, variant: str = "ewainit"):
    """Unrolled forward.  alpha: EWAInit [T] (entry t-1 at iteration t), Momentum [T, 2]
    (step, decay of iteration t in row t-1); prior: [n, 3], synd: [shots, m] {0,1}, err:
    [shots, n] Pauli codes.  Returns (loss, Q^{(T)} [shots, n, 3])."""
    if variant not in ("ewainit", "momentum"):
        raise ValueError(f"unrolled reference: variant {variant}")
    synd = torch.as_tensor(np.asarray(synd), dtype=F64)
    err = np.asarray(err, np.uint8)
    shots = synd.shape[0]
    pi0 = prior.reshape(1, 3 * tg.n)

    def clampC(x):
        return torch.clamp(x, -clamp, clamp)

    # initialisation (eq. init): m^{(0)}_{v->c} = lambda_{H_cv}(Pi^{(0)}_v)
    m_vc = clampC(lam(tg, pi0.expand(shots, -1)))
    check_sign = 1.0 - 2.0 * synd[:, tg.check]          # (-1)^{s_c} per edge
    Q_prev = pi0.expand(shots, -1)                       # Q^{(0)} = Pi^{(0)}
    g = torch.zeros(shots, 3 * tg.n, dtype=F64)          # Momentum: g^{(0)} = 0
    Q = None
    for t in range(1, T + 1):
        # horizontal update (eq. h_update): sign and phi-sum over the other edges of the check
        f = torch.cat([phi(m_vc.abs()), torch.zeros(shots, 1, dtype=F64)], dim=1)
        sg = torch.cat([torch.sign(m_vc), torch.ones(shots, 1, dtype=F64)], dim=1)
        S = f[:, tg.others[:, 0]] + f[:, tg.others[:, 1]] + f[:, tg.others[:, 2]]
        sgn = check_sign * sg[:, tg.others[:, 0]] * sg[:, tg.others[:, 1]] * sg[:, tg.others[:, 2]]
        m_cv = clampC(sgn * phi(S))
        M = m_cv @ tg.A
        if variant == "ewainit":
            # EWA prior (eq. EWAInit): Pi^{(1)} = Pi^{(0)}, Pi^{(t)} = alpha_t Pi^{(0)} + (1 - alpha_t) Q^{(t-1)}
            pit = pi0 if t == 1 else alpha[t - 1] * pi0 + (1.0 - alpha[t - 1]) * Q_prev
            # posterior (eq. p_update): Q^{(t)} = Pi^{(t)} + M^{(t)}
            Q = pit + M
        else:
            # momentum (eqs. mombp1, mombp2; the gradient of eq. mombp3 is Q^{(t-1)} - Pi - M^{(t)})
            g = alpha[t - 1, 1] * g + (1.0 - alpha[t - 1, 1]) * (Q_prev - pi0 - M)
            Q = Q_prev - alpha[t - 1, 0] * g
        if t < T:
            # vertical update (eq. v_update): m_{v->c} = lambda_{H_cv}(Q_v) - m_{c->v}
            m_vc = clampC(lam(tg, Q) - m_cv)
        Q_prev = Q
    Q3 = Q.reshape(shots, tg.n, 3)
    lse = torch.logsumexp(torch.cat([torch.zeros(shots, tg.n, 1, dtype=F64), -Q3], dim=2), dim=2)
    idx = np.zeros(err.shape, np.int64)
    for code, k in Q_INDEX.items():
        idx[err == code] = k
    q_e = torch.gather(Q3, 2, torch.as_tensor(idx).unsqueeze(2)).squeeze(2)
    q_e = torch.where(torch.as_tensor(err == 0), torch.zeros((), dtype=F64), q_e)
    return (lse + q_e).mean(), Q3


def loss_and_grad(hx, hz, alpha, prior, synd, err, T: int, clamp: float = 30.0, tg: Tanner = None,
                  variant: str = "ewainit"):
    """Loss and its gradient with respect to the per-iteration parameters (alpha [T] for
    EWAInit, [T, 2] for Momentum) and prior [n, 3] (float64 numpy)."""
    tg = tg or Tanner(hx, hz)
    a = torch.tensor(np.asarray(alpha, np.float64), requires_grad=True)
    p = torch.tensor(np.asarray(prior, np.float64).reshape(tg.n, 3), requires_grad=True)
    loss, Q = forward(tg, a, p, synd, err, T, clamp, variant)
    loss.backward()
    # alpha is not used at all when T = 1 (alpha_1 is unused): its gradient is then 0
    ga = a.grad.numpy().copy() if a.grad is not None else np.zeros(a.shape)
    return float(loss.detach()), ga, p.grad.numpy().copy(), Q.detach().numpy()


def soft_loss(q, err):
    """The same loss from a posterior q [shots, n, 3] (numpy): for finite differences."""
    q = np.asarray(q, np.float64)
    err = np.asarray(err, np.uint8)
    z = np.concatenate([np.zeros(q.shape[:2] + (1,)), -q], axis=2)
    lse = np.logaddexp.reduce(z, axis=2)
    q_e = np.zeros(err.shape)
    for code, k in Q_INDEX.items():
        q_e = np.where(err == code, q[:, :, k], q_e)
    return float((lse + q_e).mean())
