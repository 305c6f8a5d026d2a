"""Generic Levenberg-Marquardt loop (test infrastructure, FP64).

Each iteration (Background, Eq. 3-6) linearises the residuals, solves the
damped normal equations (J^T W J + lambda D^T D) dx = -J^T W r, and evaluates
the cost at x + dx.  The paper leaves the acceptance test and the damping
update unspecified; the readings used here (and by the GPU solver) are:

  * one "iteration" (trial) = one linear solve + one cost evaluation, accepted
    or not; the linearisation is recomputed only after an accepted step;
  * model decrease  L = -(b^T dx + 1/2 dx^T H dx)   (undamped IRLS model);
  * accept iff L > 0 and F(x + dx) < F(x);
  * on accept: lambda *= max(1/3, 1 - (2 g - 1)^3) with gain g = (F - F') / L,
    nu = 2 (Nielsen's rule); on reject: lambda *= nu, nu *= 2;
  * stop after max_iters trials, or when an accepted step has
    (F - F') / F < tol (COST_TOL), or |dx| <= tol (|x| + tol) (STEP_TOL),
    or lambda exceeds LAMBDA_MAX (LAMBDA_OVERFLOW).

The problem object supplies cost / linearize / solve / model_decrease / step /
norm / n_free; see ba.BAProblem and dense.DenseProblem.
"""
import math

LAMBDA_MAX = 1e32

TERM_NONE = 0
TERM_MAX_ITERS = 1
TERM_COST_TOL = 2
TERM_STEP_TOL = 3
TERM_LAMBDA_OVERFLOW = 4
TERM_NUMERICAL_FAILURE = 5
TERM_NO_WORK = 6


class LMResult:
    def __init__(self, x, cost, initial_cost, log, termination):
        self.x = x
        self.cost = cost
        self.initial_cost = initial_cost
        self.log = log
        self.termination = termination

    @property
    def trials(self):
        return len(self.log)

    @property
    def accepted(self):
        return sum(1 for e in self.log if e["accepted"])


def levenberg_marquardt(problem, x0, max_iters, tol=0.0, initial_lambda=1e-4,
                        min_diag=1e-6, max_diag=1e32):
    x = x0
    F = problem.cost(x)
    if not math.isfinite(F):
        return LMResult(x, F, F, [], TERM_NUMERICAL_FAILURE)
    if problem.n_free() == 0 or max_iters <= 0:
        return LMResult(x, F, F, [], TERM_NO_WORK if problem.n_free() == 0
                        else TERM_MAX_ITERS)
    F0 = F
    lin = problem.linearize(x)
    lam = initial_lambda
    nu = 2.0
    log = []
    term = TERM_MAX_ITERS
    for _ in range(max_iters):
        dx = problem.solve(lin, lam, min_diag, max_diag)
        xn = problem.step(x, dx)
        Fn = problem.cost(xn)
        L = problem.model_decrease(lin, dx)
        dnorm = problem.norm(dx)
        xnorm = problem.norm(x)
        accepted = bool(L > 0.0 and Fn < F)
        gain = (F - Fn) / L if L != 0.0 else float("nan")
        log.append(dict(cost=F, candidate_cost=Fn, lam=lam, model_decrease=L,
                        gain=gain, accepted=accepted, step_norm=dnorm))
        stop = None
        if accepted:
            rel = (F - Fn) / F
            x = xn
            F = Fn
            lam *= max(1.0 / 3.0, 1.0 - (2.0 * gain - 1.0) ** 3)
            nu = 2.0
            if rel < tol:
                stop = TERM_COST_TOL
        else:
            lam *= nu
            nu *= 2.0
        if stop is None and dnorm <= tol * (xnorm + tol):
            stop = TERM_STEP_TOL
        if stop is None and lam > LAMBDA_MAX:
            stop = TERM_LAMBDA_OVERFLOW
        if stop is not None:
            term = stop
            break
        if accepted:
            lin = problem.linearize(x)
    return LMResult(x, F, F0, log, term)
