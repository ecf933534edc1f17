"""Plain FP64 CPU oracle of the FFT-based magnetization method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the test-suite, the smoke check of the entry module
and the CPU-baseline leg of the benchmark use it.  It shares no code with the
HIP library (no kernels, helpers, tables or constants) and imports nothing
from it.

Contents (each function cites the passage of Prigozhin & Sokolovsky,
"FFT-based solution of 2D and 3D magnetization problems in type-II
superconductivity", that it follows):

* ``film``    -- thin-film problem, Sec. 2: stream function, power law (3),
                 eq. (9) on a staggered node/edge grid, iteration (10)-(12),
                 post-processing of Sec. 2.1.
* ``bulk``    -- bulk problem, Sec. 3: Ampere/Faraday on a Yee lattice, power
                 law (13), operator Phi of eqs. (16)-(17) and iteration (18).
* ``bs23``    -- explicit Bogacki-Shampine 3(2) pair with step control, the
                 integrator family of Matlab's ode23 named in Sec. 2.2.
* ``adjoint`` -- hand-written vector-Jacobian products of the film
                 right-hand side and of the fixed-count bulk right-hand side
                 (transposes of the operators above), the frozen-step BS23
                 step and the h_z post-processing.
* ``bean``    -- Bean critical-state closed forms for the infinite strip and
                 the thin disk, the large-n limits used in Sec. 2.3.

Everything is float64 numpy, single threaded, written for readability rather
than speed.
"""
