// Solver engine instantiation: dimension 3, Taylor-Hood degree 3.
#include "engine_impl.hpp"

namespace smg {
EngineBase *make_engine_3_3() { return new EngineT<3, 3>(); }
}  // namespace smg
