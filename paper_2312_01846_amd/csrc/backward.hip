// Backward of sigma = H(h, g) v (placeholder translation unit; the kernels
// are added alongside the forward ones).
#include "sfci_internal.h"
