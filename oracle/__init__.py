"""FP64 CPU oracle for EP with TV priors (Yao, McLaughlin, Altmann, arXiv 2110.01585).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference that the GPU library is checked against.  Only the test suite, the
package's smoke check and the CPU-baseline leg of the benchmark may import it;
the product path never does, and the two share no code (only the seeded input
generators in ``synthetic.py``, which contain no EP arithmetic).

Modules
  tilted     -- moments of the 1-D tilted distributions of the gradient u
                (Laplace x Gaussian for l1-TV, Gaussian-mixture x Gaussian for
                MoG2-TV and BG-TV, Gaussian x Gaussian for the l2 check
                prior), Sec. III-C, Eq. (marginal_tilted_un).
  operators  -- H, H^T, H^T H for identity / periodic blur / masked DFT /
                subsampled Paley-ordered Walsh-Hadamard, the spectra, and
                dense matrices for tiny problems.
  ep         -- colour classes (Fig. 1, Eq. (prior1)), site state, the
                likelihood-site update (Eqs. (tilted_P_1), (update_q0_x)),
                the TV-site update (Eq. (update_qk_x) with the Gehre-Jin
                projection), the final gather (Eq. (Q_x_final)), Algorithm 1
                and the fast EP-EM of Algorithm 2 (lambda = N / a_bar_u).
  brute      -- exact posterior marginals of tiny (3x3) denoising problems by
                grid sum-product, used to check EP approximation quality.
  convnet    -- FP64 reference of the warm-start conv net (forward/backward).

Parity status of each function is stated in its module header.
"""
