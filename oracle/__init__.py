"""ORACLE — test infrastructure, not part of the product.

A plain, slow, FP64 CPU implementation of what the matrix-free path computes, written from the paper
("Spin Hamiltonian as Matrix-Free Linear Map") and sharing no code with the HIP library:

* ``kron``     : the plain definition, H as a sum of Kronecker products (site 0 leftmost), dense or
                 scipy-sparse, for tiny systems (Sec. I; Sec. III multiplier order).
* ``mf``       : y = H x row by row in plain C (``mf_ref.c``): each row of the Kronecker sum evaluated
                 from dense local matrices built from their closed forms (Sec. IV.A spins, App. B powers
                 and general one-site operators, App. C bosons); full vectors or sampled rows.
* ``lanczos``  : Lanczos with full CGS2 reorthogonalisation and the tridiagonal eigen solve (the
                 Krylov driver the paper cites in Sec. I; the paper gives no algorithm of its own).
* ``grad``     : the gradient of y = H(theta) x (adjoint form) and of the Rayleigh quotient.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may import
this package.  The product path never does.
"""
