// Seeding job tables, shared by the seeding kernels and the host side.
#pragma once
#include "device.h"

namespace streami {

// One seeding batch for one block (device pointers; ids, max_steps and
// t_births may be NULL); its particle i takes slot first + i, and its
// workgroups of the seeding launch start at wg0.
struct SeedJob {
  const float* xyz;
  const unsigned long long* ids;
  const int* max_steps;
  const float* t_births;
  long long first;
  long long n;
  unsigned long long auto_id0;
  int blk;
  unsigned wg0;
};
// the job table of one seeding launch travels as kernel arguments (< 4 KiB)
constexpr int SEED_JOBS = 48;
struct SeedJobs {
  SeedJob j[SEED_JOBS];
  int n_jobs;
  int default_max;
  int stride;
  float t_birth;
};

}  // namespace streami
