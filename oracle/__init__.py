"""CPU FP64 oracle — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg
may import, call or load anything in this package. It shares no code with the
GPU path (``paper_2411_15332_amd``) and never imports it.

Modules:
  gates     textbook gate matrices (FP64)
  oracle    per-gate dense state update (liboracle.c), readouts, gradients,
            Grover closed form
  ref_kron  brute-force matrix-tensor-product simulation for n <= 10
  rh        the paper's RH sign rule and RH-MVM methods (Algorithm 1), small n
"""
