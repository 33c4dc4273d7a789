"""Plain FP64 CPU oracle for the rectangular MRT lattice Boltzmann method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports this
package; only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may call it.  It shares no code with the HIP path: every table,
matrix and formula here is rebuilt from the paper (Chai, Yuan & Shi,
arXiv:2206.00366) in the plainest form that numpy allows.
"""
