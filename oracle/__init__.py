"""CPU reference implementations ("oracles") for the improved-QFT DFT.

This package is TEST INFRASTRUCTURE. Only the test suite, the smoke check in
``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` may import it,
call it, or link/run anything built from it. The GPU library never does, and the
two share no code, tables or helpers.

Contents
--------
``direct``  Oracle A: the plain O(N^2) definition of the unnormalised complex
            DFT (Pasquini, Sec. 2.1, eq. qft_0A with theta = 2*pi/N, eq. qft_0D),
            in FP64 with exact integer angle reduction.
``qft``     Oracle B: the improved-QFT recursion (Sec. 5, eight mutually
            recursive functions; Sec. 3 basic elaborations; Sec. 4 for the
            shared ``cdft``/``rdft``) in FP64 numpy, with real add/multiply
            counters (Table 2) and storage-size (ln/lk, Table 1) checks.
``qft_ref.c`` The same recursion in plain C (FP64, no contraction), used only
            as the timed CPU baseline; built by ``oracle.build``.
"""
