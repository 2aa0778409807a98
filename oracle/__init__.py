"""CPU FP64 oracle for the image-plane single-pulse search (test infrastructure).

This package is test infrastructure, not product code. Only the test suite,
the smoke check and the CPU-baseline leg of the benchmark may import it. It
shares no code with the HIP library: no kernels, headers, helpers or tables.

What it computes follows the search described in section 2.2 of the paper
(the `cerberus` pipeline): per-pixel median subtraction and noise
normalisation, incoherent de-dispersion with precomputed integer shift
indices, boxcar filtering, S/N, maximum over time with its time of arrival,
and a threshold that turns pixels into candidates (top ten by S/N, section
2.3). Readings of points the paper leaves open are listed in each function.

Modules
-------
delays    dispersion delay table (section 2.2, the t_BW delay law)
stats     robust noise statistics: median and MAD (section 2.2; section 3.2)
search    normalise, de-disperse, boxcar, S/N, max/argmax, candidates
brute     nested-loop restatement used to check `search` on tiny inputs
cnn       candidate classifier forward/backward in FP64 (section 2.3)
"""
