// Engine of one (lattice, equilibrium order, storage form) class.  This file
// is compiled once per class, with DCLBM_DIM (2 or 3), DCLBM_EQ (2 or 3) and
// DCLBM_P (0 FP64, 1 FP32, 2 FP16 storage) defined by the build, so the
// device code of the twelve classes builds in parallel.
#include "engine_impl.hpp"

#if !defined(DCLBM_DIM) || !defined(DCLBM_EQ) || !defined(DCLBM_P)
#error "DCLBM_DIM, DCLBM_EQ and DCLBM_P must be defined"
#endif

#define DCLBM_CAT2(a, b, c, d) a##b##c##_##d
#define DCLBM_CAT(a, b, c, d) DCLBM_CAT2(a, b, c, d)
#define DCLBM_FACTORY DCLBM_CAT(make_engine_d, DCLBM_DIM, DCLBM_EQ, DCLBM_P)

namespace dclbm {

Engine* DCLBM_FACTORY() { return new EngineImpl<DCLBM_DIM, DCLBM_EQ, DCLBM_P>(); }

}  // namespace dclbm
