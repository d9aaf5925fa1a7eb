"""CPU oracle for the SQP/ADMM method of "GPU-Accelerated Sequential Quadratic
Programming Algorithm for Solving ACOPF" (Li, Schanen, Kim; arXiv 2310.13143).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64 NumPy/SciPy
restatement of the paper's method, written to check the HIP implementation.
Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import it; the product library never calls it and shares no code with it.

Modules
-------
acopf   ACOPF model of Section III-A: flows, objective, constraints, Lagrangian
        Hessian of each line, primal/dual infeasibility report.
qp      QP subproblem (QPsub) with the elimination of Section III-C.
lineqp  exact minimiser of one line subproblem by enumerating active sets.
direct  direct solve of the eliminated QP (primal-dual interior point).
admm    serial two-block ADMM of Section IV-B (Algorithm 2).
sqp     multiplier recovery, step assembly, l1 merit and the trust-region SQP
        loop of Section II (Algorithm 1).

Parity status of each function is stated in its docstring; functions marked
"parity unpinned" have no check independent of themselves.
"""
