"""CPU oracle of the relightable Gaussian-avatar render path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the product path.

* ``cpu``   -- ctypes binding of ``rga_oracle.c``, the FP32 mirror of every
               step whose arithmetic decides an integer (bit-exact reference).
* ``ref64`` -- the FP64 forward in plain PyTorch CPU operations; autograd of it
               is the reference gradient.
"""
