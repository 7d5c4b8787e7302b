// Host-side planning shared by the solver and the host-only layout export (no HIP here, so
// that a plain C++ build of flatten.cpp, xplan.cpp and host_layout.cpp can be checked with
// the host sanitizers).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/cfr.h"
#include "xplan.hpp"

namespace cfr {

int set_error(int code, const std::string& msg);

// Flattens and plans every game on host threads (CFR_ELEVEL or CFR_EINVAL unless every game
// has level-pure infosets and at most 16 actions). packs: plan subtree packs where the batch
// allows them (at most 4 actions in every game).
int plan_games(const cfr_game* games, int32_t n, std::vector<ExecPlan>& plans,
               int32_t& max_actions, std::string& err, bool packs);

}  // namespace cfr
