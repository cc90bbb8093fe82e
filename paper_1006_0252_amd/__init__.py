"""MI355X population annealing with weighted averages (arXiv:1006.0252): HIP kernels behind
the C ABI of include/pa.h, a ctypes binding (pa.py) and the batched/learned-schedule drivers."""
