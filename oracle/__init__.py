"""CPU oracle for the dead-time Markov stationary-PDF method.

TEST INFRASTRUCTURE ONLY.  Plain, slow, float64 NumPy/SciPy code written from
the paper (Zhang, Weerasooriya, Chennuri, Chan, "Real-Time Markov Modeling for
Single-Photon LiDAR", arXiv 2509.20500).  Only the tests, the smoke check and
the CPU-baseline leg of the benchmark may import it; the product path never
does, and it shares no code with the HIP kernels or their host library.

Modules
-------
``dtm``          flux, cumulative flux, shift, exponent/transition matrices,
                 stationary vector (dense solve, eig, GTH, power iteration).
``elementwise``  the per-element integral form of Eq. (transition_pmf),
                 integrated numerically; used to pin Theorems 1 and 2.
``montecarlo``   a Poisson-arrival, non-paralyzable dead-time detector
                 simulator (Section 2.1); pins the model against physics.
``spectral``     second eigenvalue (magnitude and phase) and mixing steps
                 (Section 4).
``mlp``          float64 forward/backward of the warm-start network.
"""
