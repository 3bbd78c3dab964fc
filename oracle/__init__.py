"""FP64 CPU oracle for LST object building (test infrastructure only).

Only tests, the smoke check and the benchmark's CPU-baseline leg import this
package. The product library never does.
"""
