"""FP64 CPU oracle for the THC second-order-exchange (SOX) self-energy.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute anything in this package: only the test suite, the smoke check and
the benchmark's CPU-baseline leg use it.  It shares no code, tables or helpers
with the HIP library; both sides only read the same seeded inputs.

Everything is plain NumPy in float64, written to be read against the paper
(Pokhilko, Yeh, Morales, Zgid, "Tensor hypercontraction for fully
self-consistent imaginary-time GF2 and GWSOX methods"):

* ``sox``        -- the SOX self-energy four ways: the literal six-index
                    definition, the one-G-at-a-time ERI chain, the THC-basis
                    form and the paper's THC contraction sequence.
* ``energy``     -- Galitskii-Migdal dynamic energy (tau quadrature and
                    Matsubara sum), density matrix, MP2 exchange closed form.
* ``transforms`` -- Chebyshev <-> Matsubara transforms, Dyson equation and one
                    self-consistency iteration.
* ``mlp``        -- forward/backward of the warm-start residual MLP.

Readings of the paper where it is silent or garbled (each also listed in the
design notes of the repository):

* G(-tau) in the SOX expression is the value stored at the mirrored grid point,
  G(beta - tau), with the expression's leading minus kept.
* The summation indices printed under the two projection steps of the THC
  sequence are garbled; they are sums over u and over p respectively.
* All inputs are real, so complex conjugates on X are dropped.
* The dynamic energy carries a factor 1/2 (spin-orbital Galitskii-Migdal form).
* The density matrix is gamma = -G(beta^-).
"""
