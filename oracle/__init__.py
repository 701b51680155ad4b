"""Reference implementations used to check the HIP path.

TEST INFRASTRUCTURE ONLY.  Only tests, the package smoke check and the
CPU-baseline leg of the benchmark may import anything from here; the product
path never does.  Nothing here shares code with the HIP library.

* ``statevector``: plain FP64 state-vector simulator (C, OpenMP) over the gate IR.
* ``brute``: dense-unitary brute force for a handful of qubits (NumPy).
* ``carleman``: the classical Carleman-linearised D1Q3 lattice Boltzmann ODE,
  its truncated Taylor propagator and the Taylor linear system L x = b
  (NumPy / SciPy).
"""
