"""FP64 CPU oracle for the contourlet transform (CT) of CVC.

TEST INFRASTRUCTURE ONLY. This package is the plain, slow reference that the
HIP path is checked against. Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import it; the product path never does.
It shares no code with the HIP path: filters, lattice geometry, layout tables
and quantiser arithmetic are all derived again here from the paper and from
the mathematics.

What the paper fixes (section 2.1, section 3.3-3.6):
  * the CT is a Laplacian pyramid (LP) followed by a directional filter bank
    (DFB) on every LP bandpass image, iterated on the lowpass (section 2.1,
    Fig. 1);
  * the DFB at level l splits into 2^l wedge-shaped subbands (section 2.1);
  * both LP and DFB use the Cohen-Daubechies 9-7 biorthogonal filters
    (section 2.1);
  * every LP level halves the resolution, and the output is the coarsest
    lowpass plus the directional subbands of every scale (section 3.3);
  * the lowpass is normalised to [0, 255], the coefficients are divided by a
    quantisation parameter and rounded to the nearest integer (sections
    3.4-3.6);
  * convolutions are computed with FFTs (section 3.10), i.e. periodically.

Everything the paper leaves open (boundary, normalisation, fan filters, tree
geometry, layout, rounding rule) follows one stated reading; each module
names the reading it implements.

Modules
  filters   closed-form 9-7 pair as polynomials in cos(omega)
  geometry  padding rule, level sizes, subband table and packed layout
  lp        periodic LP analysis and dual-frame synthesis
  dfb       quincunx fan filter bank (operator form) and the DFB tree
  ct        forward / inverse CT, padding, packing, adjoints
  quant     uniform quantiser / dequantiser (FP64 and FP32-emulating twin)
  matrix    explicit dense matrices of every stage, built from definitions
"""
