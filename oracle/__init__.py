"""FP64 CPU oracle for the Kalman-MPC solve (test infrastructure only).

This package is a plain, slow, obviously correct NumPy implementation of what
the library computes, written from the paper ("Optimal Inferential Control of
Convolutional Neural Networks", Vaziri & Fang):

* ``cnn``           the surrogate X_{k+1} = CNN(X_k, U_k) of Eq. (1)
* ``enks``          the single-pass matrix-variate ensemble Kalman smoother,
                    Eqs. (11)-(15) and Algorithm 1 (Kalman-MPC)
* ``philox``        the Philox4x32-10 counter-based generator (Salmon et al.,
                    SC'11) and the Box-Muller normals built on it, for the
                    seed-driven solve
* ``closed_forms``  textbook references that pin the smoother: the per-column
                    Kalman filter + Rauch-Tung-Striebel smoother and the dense
                    least-squares minimiser of the MPC cost (Theorem 1)
* ``cost``          the matrix-trace tracking cost of the problem setup

It shares no code with the HIP library and imports nothing from it.  Only the
test suite, the smoke check and the CPU-baseline leg of the benchmark may import
it; the product path never does.

Parity status: every function here is pinned by a CPU test against something
other than itself (library routines, brute force, closed forms, invariants, or
published known-answer vectors), except the nonlinear (tanh/GELU) solve as a
whole, which is pinned only through its parts.
"""
