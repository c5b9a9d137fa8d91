"""Plain, slow FP64 CPU oracle of the masked full-batch HMC path.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The product path (the
HIP library and its Python binding) never imports, links or calls it and
shares no code with it; both sides only share the seeded input generators of
the ``workloads`` package.

What it computes, in the paper's terms:
  * ``network``: the network F_Theta (MLP, or DeepONet with a dot-product
    combination), the potential U = -log[P(D|Theta) P(Theta_s)] up to an
    additive constant (Sec. 2.2 with the Gaussian prior and likelihood of
    App. C), and the gradient of U with respect to the selected subset
    Theta_s while Theta_~s stays fixed (Sec. 3.2).  The gradient is the plain
    definition: a dense back-propagated gradient of every parameter, from
    which the selected entries are taken.
  * ``hmc``: the leapfrog integrator, the Hamiltonian and the
    Metropolis-Hastings step of Algorithms 1 and 2, and the chain loop.
  * ``philox``: the counter-based Philox4x64-10 generator (Salmon et al.,
    SC'11) with Box-Muller normals, used for the momentum refresh and the
    Metropolis uniform so that both sides can draw the same numbers.
  * ``sensitivity``: the parameter sensitivities S_i^2 of Sec. 3.1 (the
    first-order variance share of each parameter around the VI mean,
    averaged over the training inputs) and the threshold rule that picks the
    sensitive subset, from explicit Jacobian rows.
  * ``predictive``: the posterior predictive mean and spread over stored
    samples, and the mean relative L2 error of a mean prediction.

Readings of points the paper leaves open (each is named where it is used):
  K = p^T M^-1 p / 2 (the text calls K the Gaussian log-density of p);
  leapfrog, kick-drift-kick; acceptance compared in log space, non-finite
  energies rejected; likelihood summed over every output entry of the full
  training set with its constant dropped; prior on the selected entries only;
  M = I unless a diagonal M^-1 is given; for vector outputs the squared
  output derivatives are summed over output entries and averaged over
  inputs; ties in the sensitivity order keep index order.

Parity status: every function here is pinned by tests in ``tests/`` against
closed forms, invariants, brute force or NumPy's own Philox stream.
"""
