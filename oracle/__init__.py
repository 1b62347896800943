"""CPU FP64 oracle -- test infrastructure only.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may import this
package. The HIP product path never imports, links or executes anything here.
"""
