"""CPU oracle for coarse-grained photon-number distributions of Gaussian states.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call, link or execute anything in this package;
only tests/, the smoke check and the CPU-baseline leg of the benchmark use it.

Plain, slow, obviously correct FP64 code written from the paper
(arXiv:2412.17742, Bulmer, Martinez-Cifuentes, Bell, Quesada):

  state.py  Gaussian-state assembly: covariance matrix, means, adjacency matrix
            A, loop vector gamma and vacuum probability (Sec. II).
  pgf.py    Generating function of the bin counts, G(w) = Pr(0) q(A, gamma, w)
            (Eq. q_d with the Lambda-blocked master theorem, Eq. Lamb_lhaf_master),
            and the wrapped distribution obtained by an explicit inverse DFT over
            a roots-of-unity grid (the finite-difference sieve of Sec. V with
            roots-of-unity nodes).
  lhaf.c    Brute-force loop hafnian of a matrix with repeated rows/columns
            (Eq. gen_loop_haf_def / lhaf_def), by recursion over single-pair
            matchings.
  brute.py  Exact box probabilities by summing fine-grained Fock probabilities
            (Eq. gbs_probability_distribution) over every compatible pattern
            (Eq. coarse_grained_prob, first line; Eq. prob_internal_modes).
  grad.py   Gradients of the wrapped distribution through torch autograd (CPU,
            complex128) over the same formulas.

Pinned by tests/test_oracle_*.py against closed forms, brute force, invariants
and the Fock-heralding fidelities printed in Sec. VIII A.  Parity unpinned:
none of the functions above (every one has at least one independent pin).
"""
