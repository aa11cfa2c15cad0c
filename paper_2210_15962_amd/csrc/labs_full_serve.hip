// labs_full_serve.hip -- the serving forms of the whole-space batch kernels
// (walks that pause and resume across launches; see labs_full.hip), built as
// a translation unit of their own so that they compile in parallel with the
// rest of labs_full.hip.
#define LABS_FULL_SERVING_ONLY 1
#include "labs_full.hip"
