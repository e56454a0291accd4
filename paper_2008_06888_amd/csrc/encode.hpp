// Host encoding of a plan's energy passes into device descriptors.
#pragma once
#include <string>
#include <vector>

#include "device.hpp"
#include "plan.hpp"

namespace tt {

struct EnergyProgram {
  std::vector<DevPass2> passes;
  std::vector<DevStage> stages;
  std::vector<FOp> fops;
  std::vector<BCand> cands;
  std::vector<BTerm> terms;
  std::vector<uint8_t> final_pos;   // slot -> address bit of the final state
  std::vector<BChunk> chunks;       // backward: pass runs staged in LDS together (last run first)
  int max_cand = 0;
};

// Returns "" or an error message.
std::string encode_energy(const Plan& p, const std::vector<Pass>& passes, EnergyProgram& out);

}  // namespace tt
