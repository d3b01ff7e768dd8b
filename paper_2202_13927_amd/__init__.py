"""MI355X-native closed-loop virtual clinical trials (hot path of arXiv 2202.13927).

The compute path is the HIP library built from ``csrc/``; ``vct`` is its thin
ctypes binding. Importing the package loads nothing; the binding loads the
library on first use and raises if it is missing.
"""
