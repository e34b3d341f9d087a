"""Plain FP64 CPU oracle for the preconditioned primal-dual (PPD) imaging path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, table,
constant generator or helper with the HIP library; the only common module is
``synth`` (seeded random inputs, no method arithmetic).

Modules (each function cites the passage of Onose, Dabbech & Wiaux 2017,
"An accelerated splitting algorithm for radio-interferometric imaging: when
natural and uniform weighting meet", that it follows):

* ``nufft``   -- measurement operator Phi = Theta G F Z and its adjoint (Sec. 2);
* ``sara``    -- SARA dictionary: Dirac + Daubechies 1..8 (Sec. 5.1);
* ``prox``    -- P_C, soft-threshold, P_B (Sec. 3.3), Algorithm 2 and the
                 exact metric-U proximity operator it approximates (Sec. 4.1);
* ``ppd``     -- Algorithm 3 (PPD; PD when U = I) and the SNR metric (Sec. 5);
* ``problem`` -- problem assembly: visibilities, noise level, l2 bounds,
                 uniform-weighting preconditioner, operator norm (Sec. 4.3, 5.1).

Every function is pinned by a CPU test against something other than itself
(a closed form, a brute-force evaluation, an invariant or a special case);
see the ``test_oracle_*`` modules.
"""
