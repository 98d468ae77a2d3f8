"""CPU oracle for the SBCI sigma/solve hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import anything from this package.  The product library
(``paper_2603_06101_amd``) never imports, links or calls it, and this package
never imports the product: the two share only the seeded input generators in
``workloads``.

Contents (each module cites the passage of the paper it follows):

* ``strings``      -- alpha/beta occupation strings, lexical addressing and
                      single-excitation tables written out from the
                      second-quantised definitions (brute force on bit masks).
* ``hamiltonian``  -- the determinant-basis Hamiltonian H of the paper's
                      problem statement (Results, "SBCI1 algorithm"), built
                      twice and independently: operator-by-operator
                      application and the Slater-Condon rules; its diagonal D;
                      <S^2>.
* ``sigma``        -- sigma = H c in the string basis, row by row from the
                      Slater-Condon rules (plain C, ``csrc/sigma_ref.c``, built
                      with gcc on first use), plus sampled rows.
* ``sbci``         -- SBCI1 step by step (Algorithm 1 with Sections S1.1-S1.5)
                      and a block Davidson reference, both in FP64 NumPy.
* ``sbci2``        -- SBCI2 step by step (Algorithm 2 with Sections S2.1-S2.5).
* ``symmetry``     -- the irrep block layout of a point-group symmetric
                      problem and the blocked sigma as the restriction of the
                      full sigma.

Pins: see ``tests/test_oracle_*.py``.  Functions whose results the paper does
not fix and that no closed form or brute force checks are marked
"parity unpinned" in their docstrings.
"""
