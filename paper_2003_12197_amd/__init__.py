"""HERS encrypted search on MI355X.

libhers.so (built from csrc/ by build.py) implements the path; hers_gpu is its
Python binding and synth the seeded synthetic workloads.
"""
