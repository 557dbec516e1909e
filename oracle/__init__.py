"""CPU oracle for the encrypted FFT -- TEST INFRASTRUCTURE ONLY.

A plain, slow, independent implementation of what the accelerated path
computes: the fixed-point FFT as integers (fixedpoint), the canonical gate
netlist with its noise bound (netlist), SplitMix64 (prng), packed GSW13 over
q = 2^k in plain C (gsw, gsw_ref.c), textbook GSW13 with explicit Flatten
for tiny parameters (literal_gsw) and ring-GSW over Z_p[X]/(X^d + 1) with
negacyclic products by their definition (rgsw, rgsw_ref.c).

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
or execute anything in this package.  It shares no code with the HIP library.
"""
