// Library-internal access to a context's tunable settings (the autotuner
// saves them, changes them while it measures, and restores them).
#pragma once

#include "../../include/sg.h"

struct SgSettings {
  int device;
  int wgs_per_cu;
  int resume_spacing;
  int graphs;
  int grid;
};
SgSettings sg_settings_get(const sg_ctx* ctx);
void sg_settings_set(sg_ctx* ctx, const SgSettings& s);
// Sets the calling thread's sg_last_error message and returns `code`.
sg_status sg_fail(sg_status code, const char* msg);
