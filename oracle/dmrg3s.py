"""DMRG3S sweep driver (oracle; test infrastructure only).

Follows the site update of Sec. 5 step by step (left-to-right shown there,
right-to-left mirrored as in Sec. 4.1):
  1. smallest eigenpair (lambda*, M*) of H_eff = L_{i-1} R_{i+1} W_i,
  2. expansion term P_i = alpha L_{i-1} M* W_i (alpha R_{i+1} M* W_i),
  3. M~ = [M* P] ([M*; P]); the neighbour is zero-padded implicitly,
  4. SVD of M~ and truncation of the expanded bond,
  5. S V^T (U S) multiplied into the neighbour, which is renormalised,
  6. the new environment L_i (R_i),
  7. the energy E_f of the neighbour after truncation and the alpha update
     of Sec. 6,
  8. move on.

Readings of points the paper leaves open (shared with the GPU path as data,
not code):
  * eigensolver: Lanczos with full re-orthogonalisation, warm-started from
    the current tensor, residual <= 1e-12 max(1, |lambda|);
  * truncation target: min(mmax, d^b, d^(l-b)) per bond b, dropping
    singular values s_j <= eps s_0 (eps = 1e-14);
  * the neighbour is renormalised after step 5, so E_f is a Rayleigh quotient;
  * E_before of the next site is E_f of this one;
  * alpha rule (Sec. 6 keeps dE_T near -0.3 dE_O): with dE_O = lambda* -
    E_before and dE_T = E_f - lambda*: if the truncation discarded no weight
    (discarded <= 1e-12 of ||M~||^2) the enrichment had no effect on the
    state and alpha is left unchanged; elif |dE_O| < 1e-13 |E| shrink alpha
    by 0.8; elif dE_T < 0.3 |dE_O| (including dE_T < 0) grow it by 1.25;
    else shrink it by 0.8; alpha is kept in [1e-16, 1];
  * expansion="residual" replaces P by the exact residual H Psi - E Psi
    (the Sec. 4 opening), with E the eigenvalue lambda* of step 1, its far
    side projected onto the current basis and its near side exact (see
    contract.residual_expanded_l2r); its right-side vectors are written on
    an orthonormal basis of their span (metric eigenvalues at or below
    n u lambda_max are exact linear dependences), and the expanded tensor is
    then truncated by the same SVD and the same eps rule as the cheap term;
  * one sweep is right-to-left over sites l..2 followed by left-to-right over
    sites 1..l-1 (the initial state is left-canonical with its centre on
    site l); E_s is the last lambda* of sweep s and the run stops when
    |E_s - E_{s-1}| / |E_s| < tol.
"""
import numpy as np

from . import contract as C
from .lanczos import lanczos_ground
from .mps import bond_budget, left_canonicalize

ALPHA_TARGET = 0.3
ALPHA_GROW = 1.25
ALPHA_SHRINK = 0.8
ALPHA_STALL = 1e-13
ALPHA_NO_CUT = 1e-12
ALPHA_MIN = 1e-16
ALPHA_MAX = 1.0


class DMRG3S:
    def __init__(self, mpo, tensors, mmax, alpha0=1e-3, eps=1e-14,
                 lanczos_tol=1e-12, lanczos_kmax=40, adaptive_alpha=True, expansion="heuristic"):
        if expansion not in ("heuristic", "residual"):
            raise ValueError("expansion must be 'heuristic' or 'residual'")
        self.expansion = expansion
        self.W = [np.asarray(w, dtype=np.float64) for w in mpo]
        self.l = len(mpo)
        self.d = self.W[0].shape[2]
        self.eps = eps
        self.tol = lanczos_tol
        self.kmax = lanczos_kmax
        self.adaptive = adaptive_alpha
        self.alpha = float(alpha0)
        self.budget = bond_budget(self.l, self.d, mmax)
        self.M = left_canonicalize(tensors)
        l = self.l
        self.Lenv = [None] * (l + 1)
        self.Renv = [None] * (l + 1)
        self.Lenv[0] = np.ones((1, 1, 1))
        for i in range(l - 1):
            self.Lenv[i + 1] = C.update_left(self.Lenv[i], self.W[i], self.M[i])
        self.Renv[l] = np.ones((1, 1, 1))
        if expansion == "residual":
            # environments of the channel pairs of H^2 (metric of the residual)
            self.H2L = [None] * (l + 1)
            self.H2R = [None] * (l + 1)
            self.H2L[0] = np.ones((1, 1, 1, 1))
            for i in range(l - 1):
                self.H2L[i + 1] = C.update_left_h2(self.H2L[i], self.W[i], self.M[i])
            self.H2R[l] = np.ones((1, 1, 1, 1))
        self.E_before = C.energy(self.Lenv[l - 1], self.W[l - 1], self.Renv[l], self.M[l - 1])
        self.history = []
        self.sweep_energies = []

    # --- pieces -----------------------------------------------------------
    def eigensolve(self, i):
        L, W, R = self.Lenv[i], self.W[i], self.Renv[i + 1]
        lam, x, nmv, ok = lanczos_ground(lambda v: C.apply_heff(L, W, R, v), self.M[i],
                                         tol=self.tol, kmax=self.kmax)
        return lam, x, nmv

    def update_alpha(self, lam, Ef, discarded, total_weight):
        if not self.adaptive:
            return
        dEO = lam - self.E_before
        dET = Ef - lam
        if discarded <= ALPHA_NO_CUT * total_weight:
            pass
        elif abs(dEO) < ALPHA_STALL * abs(lam):
            self.alpha *= ALPHA_SHRINK
        elif dET < ALPHA_TARGET * abs(dEO):
            self.alpha *= ALPHA_GROW
        else:
            self.alpha *= ALPHA_SHRINK
        self.alpha = min(ALPHA_MAX, max(ALPHA_MIN, self.alpha))

    def _record(self, i, direction, lam, Ef, k, disc, nmv):
        self.history.append(dict(site=i, dir=direction, E_before=self.E_before, lam=lam,
                                 E_f=Ef, alpha=self.alpha, k=k, discarded=disc, matvecs=nmv))

    def step_r2l(self, i):
        lam, psi, nmv = self.eigensolve(i)
        if self.expansion == "residual":
            Mt = C.residual_expanded_r2l(self.Lenv[i], self.W[i], self.Renv[i + 1], self.H2L[i], psi, lam,
                                         self.alpha)
        else:
            P = C.expansion_term_r2l(self.Renv[i + 1], self.W[i], psi, self.alpha)
            Mt = C.expanded_tensor_r2l(psi, P)
        B, A, s, disc = C.truncate_r2l(Mt, psi, self.M[i - 1], self.budget[i], self.eps)
        A = A / np.linalg.norm(A)
        self.M[i] = B
        self.M[i - 1] = A
        self.Renv[i] = C.update_right(self.Renv[i + 1], self.W[i], B)
        if self.expansion == "residual":
            self.H2R[i] = C.update_right_h2(self.H2R[i + 1], self.W[i], B)
        Ef = C.energy(self.Lenv[i - 1], self.W[i - 1], self.Renv[i], A)
        self._record(i, "r2l", lam, Ef, B.shape[0], disc, nmv)
        self.update_alpha(lam, Ef, disc, float(np.sum(s ** 2)))
        self.E_before = Ef
        return lam

    def step_l2r(self, i):
        lam, psi, nmv = self.eigensolve(i)
        if self.expansion == "residual":
            Mt = C.residual_expanded_l2r(self.Lenv[i], self.W[i], self.Renv[i + 1], self.H2R[i + 1], psi, lam,
                                         self.alpha)
        else:
            P = C.expansion_term_l2r(self.Lenv[i], self.W[i], psi, self.alpha)
            Mt = C.expanded_tensor_l2r(psi, P)
        A, B, s, disc = C.truncate_l2r(Mt, psi, self.M[i + 1], self.budget[i + 1], self.eps)
        B = B / np.linalg.norm(B)
        self.M[i] = A
        self.M[i + 1] = B
        self.Lenv[i + 1] = C.update_left(self.Lenv[i], self.W[i], A)
        if self.expansion == "residual":
            self.H2L[i + 1] = C.update_left_h2(self.H2L[i], self.W[i], A)
        Ef = C.energy(self.Lenv[i + 1], self.W[i + 1], self.Renv[i + 2], B)
        self._record(i, "l2r", lam, Ef, A.shape[2], disc, nmv)
        self.update_alpha(lam, Ef, disc, float(np.sum(s ** 2)))
        self.E_before = Ef
        return lam

    # --- driver -----------------------------------------------------------
    def sweep(self):
        lam = None
        for i in range(self.l - 1, 0, -1):
            lam = self.step_r2l(i)
        for i in range(0, self.l - 1):
            lam = self.step_l2r(i)
        self.sweep_energies.append(lam)
        return lam

    def run(self, tol=1e-12, max_sweeps=50, min_sweeps=2):
        prev = None
        for s in range(max_sweeps):
            E = self.sweep()
            if prev is not None and s + 1 >= min_sweeps and abs(E - prev) / abs(E) < tol:
                return E, s + 1
            prev = E
        return self.sweep_energies[-1], max_sweeps

    def bond_dims(self):
        return [1] + [t.shape[2] for t in self.M]
