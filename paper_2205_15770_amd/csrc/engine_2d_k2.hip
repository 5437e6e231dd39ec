// Solver engine instantiation: dimension 2, Taylor-Hood degree 2.
#include "engine_impl.hpp"

namespace smg {
EngineBase *make_engine_2_2() { return new EngineT<2, 2>(); }
}  // namespace smg
