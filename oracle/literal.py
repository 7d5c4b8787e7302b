"""The paper's matrix formulation of CFR, evaluated with dense numpy matrices.

Test infrastructure (oracle): not part of the product path. For tiny games only.

Everything follows Section 3 as printed, with node ids as matrix indices:

Setup (Section 3.1)
  G[v, v']       = 1 iff v = parent(v')                      tree adjacency
  L^(l)[v, v']   = 1 iff v = parent(v') and depth(v') = l    level graphs, l = 1..D
  M^(Q+,V)[q, v] = 1 iff q = (f_h(parent(v)), f_a(v))       node -> incoming rational pair
  M^(H+,Q+)[h, q] = 1 iff q = (h, a) for some a              pair -> infoset
  M^(V,I+)[v, i] = 1 iff player i acts at parent(v)           node -> acting player
  s^(sigma0)[v]  = sigma_0 of the chance edge into v, else 0
  sigma^(T=1)    = 1 / (M^(H+,Q+)^T (M^(H+,Q+) 1))             uniform strategy

Iteration (Section 3.2)
  s      = M^(Q+,V)^T sigma + s^(sigma0)
  U^(D+1) = terminal payoffs; U^(l) = (L^(l) (.) S) U^(l+1) + U^(l+1)    (Eq. expected_payoffs_matrix_recurrence)
  Pi^(0) = 1_{v=v0}; Pi^(l) = (L^(l)^T Pi^(l-1)) (.) Scheck + Pi^(l-1)      (Eq. excepted_reach_probabilities_matrix_recurrence)
  Scheck[v, i] = s_v unless player i acted into v (then 1); Shat is the complement (Eq. strategies_matrix)
  picheck = (M^(V,I+) (.) Pi^(D)) 1;  pihat likewise with Shat
  pibar = M^(H+,Q+) M^(Q+,V) pihat;  pibar_sum = pibar_sum' + pibar
  sigmabar = sigmabar' + (M^(H+,Q+)^T (pibar / pibar_sum)) (.) (sigma - sigmabar')   (Eq. average_strategy_profile_vector)
  rtilde = M^(Q+,V) (picheck (.) ((M^(V,I+) (.) (U - G^T U)) 1))
  rbar = rbar' + (rtilde - rbar') / T                                       (Eq. average_counterfactual_regrets_vector)
  rbar_plus_sum = M^(H+,Q+)^T (M^(H+,Q+) rbar^+)
  sigma' = rbar^+ / rbar_plus_sum where that sum > 0, else sigma^(T=1)

Where pibar_sum is 0 the printed update divides 0 by 0; it is read as keeping
sigmabar' (which starts uniform), i.e. a uniform average strategy until some
weight arrives.
"""
from __future__ import annotations

import numpy as np

from .tree import Tree


class Literal:
    def __init__(self, tree: Tree):
        self.tree = tree
        n = tree.n
        V = n
        D = max(tree.depth)
        self.D = D
        Q = tree.Q
        Hs = tree.rational
        self.G = np.zeros((V, V))
        self.L = [None] + [np.zeros((V, V)) for _ in range(D)]
        self.MQV = np.zeros((Q, V))
        self.MHQ = np.zeros((len(Hs), Q))
        self.MVI = np.zeros((V, 2))
        self.s0 = np.zeros(V)
        hrow = {h: r for r, h in enumerate(Hs)}
        for h in Hs:
            for a in range(tree.nact[h]):
                self.MHQ[hrow[h], tree.qoff[h] + a] = 1.0
        for v in range(n):
            for a, c in enumerate(tree.children[v]):
                self.G[v, c] = 1.0
                self.L[tree.depth[c]][v, c] = 1.0
                h = tree.infoset[v]
                pl = tree.player[h]
                if pl == 0:
                    self.s0[c] = tree.sigma0[h][a]
                else:
                    self.MQV[tree.qoff[h] + a, c] = 1.0
                    self.MVI[c, pl - 1] = 1.0
        self.U_terminal = np.zeros((V, 2))
        for v in range(n):
            if tree.is_terminal(v):
                self.U_terminal[v, 0] = tree.u1[v]
                self.U_terminal[v, 1] = -tree.u1[v]
        ones = np.ones(Q)
        self.sigma1 = ones / (self.MHQ.T @ (self.MHQ @ ones))

    def iterate(self, sigma, rbar_prev, sigmabar_prev, pibar_sum_prev, T: int) -> dict:
        """One iteration at 1-based iteration number T, using strategy ``sigma``."""
        t = self.tree
        D = self.D
        s = self.MQV.T @ sigma + self.s0
        U = self.U_terminal.copy()                       # U^(D+1)
        for l in range(D, 0, -1):
            LS = self.L[l] * s[None, :]                  # L^(l) (.) S, S[v, v'] = s_v'
            U = LS @ U + U
        Scheck = np.where(self.MVI == 0, s[:, None], 1.0)
        Shat = np.where(self.MVI == 1, s[:, None], 1.0)
        Pi = np.zeros((t.n, 2))
        Pi[t.root, :] = 1.0
        Ph = Pi.copy()
        for l in range(1, D + 1):
            Pi = (self.L[l].T @ Pi) * Scheck + Pi
            Ph = (self.L[l].T @ Ph) * Shat + Ph
        picheck = (self.MVI * Pi).sum(axis=1)
        pihat = (self.MVI * Ph).sum(axis=1)
        pibar = self.MHQ @ (self.MQV @ pihat)
        pibar_sum = pibar_sum_prev + pibar
        ratio = np.divide(pibar, pibar_sum, out=np.zeros_like(pibar), where=pibar_sum != 0)
        sigmabar = sigmabar_prev + (self.MHQ.T @ ratio) * (sigma - sigmabar_prev)
        diff = U - self.G.T @ U
        rtilde = self.MQV @ (picheck * (self.MVI * diff).sum(axis=1))
        rbar = rbar_prev + (rtilde - rbar_prev) / T
        rplus = np.maximum(rbar, 0.0)
        rsum = self.MHQ.T @ (self.MHQ @ rplus)
        sigma_next = np.where(rsum > 0, np.divide(rplus, rsum, out=np.zeros_like(rplus),
                                                  where=rsum > 0), self.sigma1)
        return {"s": s, "U": U, "Pi_check": Pi, "Pi_hat": Ph, "picheck": picheck,
                "pihat": pihat, "pibar": pibar, "pibar_sum": pibar_sum, "sigmabar": sigmabar,
                "rtilde": rtilde, "rbar": rbar, "sigma_next": sigma_next}

    def run(self, iterations: int) -> dict:
        Q = self.tree.Q
        sigma = self.sigma1.copy()
        rbar = np.zeros(Q)
        sigmabar = self.sigma1.copy()
        pibar_sum = np.zeros(self.MHQ.shape[0])
        out = None
        for T in range(1, iterations + 1):
            out = self.iterate(sigma, rbar, sigmabar, pibar_sum, T)
            sigma, rbar, sigmabar, pibar_sum = (out["sigma_next"], out["rbar"], out["sigmabar"],
                                                out["pibar_sum"])
        return out
