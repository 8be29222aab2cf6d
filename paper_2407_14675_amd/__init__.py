"""MI355X-native semi-Lagrangian dynamic programming for planar low-thrust
orbit transfer (arXiv 2407.14675, Section 3).

The compute path is the HIP library `libdpo.so` (C ABI declared in
include/dpo.h); `paper_2407_14675_amd.dpo` is its thin Python binding.  This
package file imports nothing heavy so that the input generators
(`paper_2407_14675_amd.inputs`) can be used without the device library.
"""
