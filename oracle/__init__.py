"""Oracle: a plain, slow, obviously correct CPU implementation of the
steady-state method, in complex128 (numpy / scipy).

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` use it.  It shares no code with the
HIP library (``paper_1411_4356_amd``); the only thing both read is the seeded
parameter module ``workloads``.

Modules
-------
model     -- operators, Hamiltonian Eq. (1), Liouvillian Eq. (3)-(4) by
             Kronecker products, trace-constrained system Eq. (5), weight w.
direct    -- direct solve of Eq. (5), normalisation, observables.
ordering  -- bandwidth/profile (Sec. II) and Cuthill-McKee / RCM (Sec. III).
ilut      -- dual-threshold incomplete LU (Sec. II) and its application.
levels    -- level schedule (dependency depth) of triangular factors.
adjoint   -- gradients of observables by the adjoint of Eq. (5).

Parity status of each function is stated in its docstring; functions with no
independent pin say "parity unpinned".
"""
