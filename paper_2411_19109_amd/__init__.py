"""MI355X-native level-set LLG forward/adjoint path (HIP, gfx950).

Importing the package loads nothing; ``paper_2411_19109_amd.llg`` loads the
HIP library on first use and fails loudly when it has not been built.
"""
