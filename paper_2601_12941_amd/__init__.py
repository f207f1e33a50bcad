"""MI355X-native reliability-guided 2D DIC (IC-GN on ZNSSD, cubic B-spline
interpolation, frontier-wave propagation).  The compute path is the HIP
library built from csrc/; `dic` is its Python binding."""
