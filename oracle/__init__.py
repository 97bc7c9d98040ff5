"""FP64 CPU oracle of the particle-mesh gravity step with linear-response neutrinos.

TEST INFRASTRUCTURE ONLY. Nothing in the product path imports this package: only the
tests, the smoke check and the benchmark's CPU-baseline leg may use it. It shares no
code, headers, tables or constants with the HIP library; both sides read only the seeded
inputs made by ``synth``.

It is a plain, slow, step-by-step FP64 NumPy implementation of the method of
Ali-Haimoud & Bird (arXiv:1209.0461), written to be checked against the paper by eye:

  background  Sec. 2.1 constants, flat matter+Lambda H(a), superconformal time (Sec. 3.2)
  kernel      the free-streaming kernel I(x): the fit eq. (fit) and series of Appendix C
  pm          cloud-in-cell deposit, FFT, k-binning of P_cdm, rescaling by the neutrino
              response (eq. (phases) and the total-matter sum of Sec. 4.3 (iv)),
              Poisson's equation (eq. (Poisson)), spectral gradient, inverse FFT and
              cloud-in-cell interpolation
  response    the neutrino amplitude P_nu^{1/2}(k, tau) of eq. (P-final), by quadrature
              over the stored history, with the single-iteration rule of Sec. 4.3 (iii)
              and Appendix B
  step        one full step in the order of Sec. 4.3 (ii)-(iv)
  mlp         an FP64 reference of the small surrogate network (not from the paper)

Pins (tests marked "not gpu") tie every function to something other than itself: closed
forms, the paper's printed numbers and limits, invariants and brute force.
"""
from . import background, kernel, pm, response, step, mlp  # noqa: F401
