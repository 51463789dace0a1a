"""FP64 CPU oracle of one SIPF-W time step (Hu, Wang, Xin, Zhang, "A Novel Stochastic
Particle-Field Algorithm for a Reaction-Diffusion-Advection Cancer Invasion Model").

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously-correct restatement of
the method in numpy float64.  Only the test suite, the smoke check of the build entry point
and the CPU-baseline leg of the benchmark may import it.  The GPU library never calls it and
shares no code with it: no kernels, helpers, tables or constants.

Modules
-------
philox     counter-based Philox4x32-10 generator (Salmon et al., SC'11) and Box-Muller
           normals, the Wiener increments of the Euler-Maruyama update (eq. u_hat_update).
pic        particle-in-cell transfers: trilinear assignment R_h and interaction kernel
           K_h = h^3 R_h (Sec. 2.2.1-2.2.2, Alg. p2g and Alg. g2p), and the fourth-order
           assignment R_h^(4).
spectral   Fourier wavenumbers, the implicit (backward-Euler) diffusion-decay multiplier
           (eq. k_q_tilde_update), the exponential and aliased multipliers (eq. k_q_update,
           Lemma kernel), the low-pass filter and the spectral gradient (eq. gradv).
step       one step of Alg. sipf-pic with the readings listed in the design notes, plus the
           diagnostics (Lemma mass, Corollary mass, positivity lemma).
resample   residual resampling (Alg. res_res).

Parity status
-------------
Every function here is pinned by a CPU test against something other than itself (closed
forms, brute force on tiny inputs, a library implementation), except where a module header
says "parity unpinned".
"""
