"""TEST INFRASTRUCTURE -- NOT PART OF THE PRODUCT.

Plain CPU oracle of range-filtered k-NN over HSIG: the exact FP64 definition
(``exact``) and the paper's index build and search (``hsig``).  Only the tests,
the smoke check and the CPU-baseline leg of the benchmark may import it.
"""
