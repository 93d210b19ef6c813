"""MI355X state-vector simulator for deep circuits with gate fusion and
mid-circuit measurement (arXiv:2310.17739).

The simulation runs in ``libqsim.so`` (C ABI in ``include/qsim.h``); the
``qsim`` module is its ctypes binding.
"""
