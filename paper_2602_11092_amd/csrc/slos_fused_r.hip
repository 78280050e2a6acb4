// The fused adjoint's instances for restricted computation spaces
// (unbunched, dual-rail; arXiv 2602.11092, Sec. II-B), built in a
// translation unit of their own so that the standard instances' code does
// not change and the two compile in parallel.  The kernels are those of
// slos_fused.hip with the marked-successor select switched on.
#define SLOS_FUSED_RESTRICTED_INSTANCES
#include "slos_fused.hip"
