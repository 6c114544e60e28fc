"""FP64 CPU oracle for hierarchical iso-surface extraction on ReLU INRs.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain, float64
reference that the HIP library is checked against.  Only the test suite, the
package smoke check and the benchmark's CPU-baseline leg may import it; the
product path never does, and this package never imports the product.  It
shares no code, tables or constants with the HIP library: its marching-cubes
table is generated here from the face-consistent rule, independently of the
library's own generator.

Method source: Li & Shen, "Improving Efficiency of Iso-Surface Extraction on
Implicit Neural Representations Using Uncertainty Propagation"
(arXiv 2402.13861).  Each function cites the section / equation / algorithm
it follows.

Modules
-------
mlp        plain MLP evaluation (Sec. III-B)
rules      activation linearisations: Chebyshev/minimax for affine
           arithmetic (Eq. 4) and Gaussian least squares for uncertainty
           propagation (Eq. 9-10, App. D ReLU, Sine and ELU rows)
propagate  layer-by-layer range analysis (Eq. 1-4), its RA-UA read-off
           (Eq. 5) and uncertainty propagation (Eq. 6-9), plus a
           covariance-form cross-check
octree     hierarchical active-cell search (Alg. 1, octree and k-d tree)
mc         marching-cubes case table (generated) and triangle emission
metrics    FPR/FNR (Sec. V-A-3) and parity helpers
surrogate  float64 forward/backward/Adam of the surrogate MLP and its
           band partition
distribution  Monte Carlo histogram of a block and the KL divergence of
           Eq. 11 from the UP, RA-UA and few-sample Gaussians (Sec. V-E)
"""
