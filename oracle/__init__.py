"""Oracle for the WENO5 / SSP-RK3 Teukolsky solver: plain, slow, FP64.

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the CPU-baseline leg
of the benchmark may import it; the product library and its Python binding
never do, and the two share no code.

* ``coefficients`` derives the chart-T coefficients symbolically from the
  Boyer-Lindquist master equation (paper Sec. 2.1-2.3).
* ``teuk_oracle.c`` is a scalar C solver (WENO5 per Sec. 3.1.2, centred theta
  differences, SSP-RK(3,3) per Sec. 3.2), driven from ``solver``.
"""
