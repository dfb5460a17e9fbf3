"""CPU FP64 oracle for the space-charge particle-in-cell step.

This package is TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run it.  The product path (the HIP library
``libpic.so`` and its Python binding ``paper_2208_02382_amd``) never imports, links or calls
anything here, and nothing here imports the product path.

What it computes (paper, section "Model Assumptions"): particles are pushed in s by linear
symplectic maps; space charge is electrostatic in the bunch rest frame, found by a Poisson solve
there, and applied by a split-operator (kick between half drifts).  The paper names the
building blocks -- charge deposition, Poisson solve, beam statistics -- and the B-spline shape
order (section "Usage Example", Listing 1), but gives no formulas for them.  Every formula
below is therefore a stated reading; each module names its reading, and the module docstrings
list which function is pinned by which test.

Modules
-------
constants  physical constants (SI 2019 exact values and CODATA 2018 eps0)
dd         double-double arithmetic (Dekker 1971, Knuth TwoSum) with log/atan/sqrt
igf        integrated Green's function of 1/r over a rest-frame cell (Qiang et al. 2006)
pic        reference particle, geometry, shapes, deposit, Hockney solve, field, gather, push,
           step, tracking, moments
rng        Philox4x32-10 (Salmon et al., SC'11) and Box-Muller, for the on-device generator
"""
