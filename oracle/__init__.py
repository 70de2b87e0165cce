"""CPU FP64 reference implementation (the oracle) -- test infrastructure only.

This package is a plain, slow, deliberately simple restatement of what the
paper's method computes:

* the curl-curl time-harmonic Maxwell problem with impedance and metallic
  boundary conditions and its bilinear weak form (Sec. 2, eq. (1)-(4));
* high-order Nedelec edge elements built from the generators
  lambda^k w^e (Sec. 3), with a fixed independent subset of them;
* the ORAS preconditioner sum_s R_s^T D_s A_s^{-1} R_s with impedance
  transmission conditions on the subdomain interfaces (Sec. 4);
* GMRES preconditioned by it, single right-hand side and multiple
  right-hand sides (Sec. 5, the pseudo-block description; block GMRES is
  the variant listed as future work in Sec. 6).

It exists to check the GPU library.  Only the test suite, the smoke entry
point and the CPU-baseline leg of the benchmark may import it; the library
itself never calls it, and it shares no code with the library.

Numbering, sign and selection conventions that the paper leaves open are
stated in each module's docstring.
"""
