"""Oracle for the D2Q37 step, the learned collide and its random draws.

TEST INFRASTRUCTURE ONLY. Plain, slow, obviously correct CPU code written
from the paper and from the mathematics it relies on. Only the tests, the
smoke check and the CPU-baseline leg of the benchmark may import it; the GPU
library and its Python binding never do, and share no code with it.
"""
