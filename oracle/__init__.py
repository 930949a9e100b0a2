"""FP64 CPU oracle for the space-VLBI FX correlator -- TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, obviously correct numpy implementation of what
the correlator computes.  Only tests, the smoke check and the CPU-baseline leg
of the benchmark may import it; the product path (the HIP library and its
binding) never does, and shares no code with it.

The paper (an FX correlator, DiFX, extended for a space antenna: Fourier
transform first, then cross-multiply; a delay model that handles a moving
antenna and the spacecraft-to-tracking-station transmission delay; data read
from a Mark5B-style recording) names the steps but prints no formulas.  The
steps below are therefore the standard FX definitions written out in the
paper's order, with every convention the paper leaves open fixed explicitly:

  O1  frame midpoint time           t_mid = (j0 + f N + N/2) / fs
  O2  delay polynomial               tau = Horner, separate multiply and add
  O3  integer / fractional delay     D = tau fs, n_int = floor(D + 1/2), d = D - n_int
  O4  frame validity                 window inside the recording, good sync words
  O5  2-bit unpack                   q[n] = level(code(stream, base + n))
  O6  fringe rotation                y[n] = q[n] exp(+2 pi i phi(t_n)), phi = nu tau (long double)
  O7  FFT to channels                Y[k] = sum_n y[n] exp(-2 pi i k n / N), k < N/2
  O8  fractional-delay correction    Y[k] *= exp(+2 pi i k d / N)
  O9  cross-multiply-accumulate      Vsum_ij[k] += Y_i[k] conj(Y_j[k]), i <= j
  O10 finalise                       V_ij = Vsum_ij / W_ij

Modules: fx (O1-O10), xf (brute-force lag-domain correlation and O(N^2) DFT).
"""
