"""CPU oracle for the superfast line-spectral-estimation path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import, call or execute anything in
this package.  The HIP library never imports it and shares no code with it.

The oracle is plain and slow on purpose: it forms the covariance densely,
Cholesky-factors it and evaluates every quantity from its definition in the
paper (Hansen, Fleury, Rao, "Superfast Line Spectral Estimation", IEEE TSP
2018), in FP64.  Each function names the section / equation it follows.

Modules
-------
numerics   -- covariance, factor (rho, delta, ln|C|), C^{-1} y, diagonal sums
              omega, active-set vectors q..x, grid q^G / s^G, derivatives,
              activation / deactivation quantities.
estimator  -- the block-coordinate-descent estimator (Sec. II-C/D/E); every
              point the paper leaves open is a field of its Params with the
              reading taken.
mmv        -- the multiple-measurement-vector model of Sec. V: its objective,
              summed derivatives, single-component criteria and beta update,
              and the estimator on them (G = 1 is the estimator above, bit for
              bit).
incomplete -- incomplete observations (Sec. IV): Phi keeps M weighted samples;
              C is M x M and every quantity is formed densely from its
              definition under Phi (every sample observed with unit weights is
              the estimator above, bit for bit).

Parity status: every numerics function is pinned by tests under
``tests/test_oracle_*.py`` (closed forms, brute force, finite differences,
independent identities).  The estimator's exact trajectory (iteration count,
activation order) is "parity unpinned" beyond agreement with the HIP path,
because the paper prints no worked example; its end results are pinned by the
statistical reproduction of the accuracy-vs-SNR experiment and by noiseless
recovery.
"""
