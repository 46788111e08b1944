"""FP64 CPU oracle of the coupled Biot LBM (test infrastructure only).

Only tests/, the smoke check and the benchmark's CPU-baseline leg import this
package; the product path (paper_2409_11382_amd) never does.
"""
