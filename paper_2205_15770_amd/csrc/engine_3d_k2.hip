// Solver engine instantiation: dimension 3, Taylor-Hood degree 2.
#include "engine_impl.hpp"

namespace smg {
EngineBase *make_engine_3_2() { return new EngineT<3, 2>(); }
}  // namespace smg
