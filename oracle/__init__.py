"""FP64 CPU oracle for smooth-surface UTD creeping-wave fields.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
GPU library is checked against.  Only ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import or run anything in here;
the product library never does, and this package imports nothing from the
product (``paper_2310_10578_amd``).

What it computes (Eqs. (1)-(4) of the paper, with the UTD coefficients that the
paper only names taken from the off-surface UTD of Pathak, Burnside and
Marhefka, IEEE Trans. AP-28(5), 1980, and Kouyoumjian and Pathak, Proc. IEEE
62(11), 1974):

* ``fock``      -- Pekeris/Fock functions p*_s, p*_h, their regular parts and
                   the transition function F(X).
* ``geometry``  -- attachment/detachment points, geodesics, divergence factors
                   and reflection points on spheres and vertical cylinders.
* ``occlusion`` -- segment any-hit tests against triangles (plain C, uniform
                   grid) and against the other bodies (closed form).
* ``field``     -- the coherent receiver field of Eqs. (1)-(4).
* ``mie``       -- exact series for a PEC sphere and a PEC circular cylinder,
                   used only to validate the oracle itself.
* ``grad``      -- reference gradients by Richardson-extrapolated central
                   differences of ``field`` with the classification frozen.
"""
