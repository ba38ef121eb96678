"""MI355X-native SPG solver for the reweighted weighted-l1 + TV density-map reconstruction
(Luo, arXiv 1905.13408).  The HIP library is loaded lazily by ``paper_1905_13408_amd.spg``."""
