// Solver engine instantiation: dimension 2, Taylor-Hood degree 3.
#include "engine_impl.hpp"

namespace smg {
EngineBase *make_engine_2_3() { return new EngineT<2, 3>(); }
}  // namespace smg
