// Progressive training schedule (Sec. 5.8, "Online training and rendering"):
// training runs in iterations whose sample counts double; it stops as soon
// as the training share of the budget is used; a finished iteration starts
// the next one only while less than half of the training budget is used,
// otherwise the current iteration keeps gathering samples until rendering
// starts; the guide is always fitted from the last iteration's samples only.
// Host-side state machine; the caller owns the clock.
#include "../../include/mpg.h"

#include <string>

mpg_status fail(mpg_status code, const std::string& msg);

extern "C" mpg_status mpg_train_init(const mpg_train_plan* plan, mpg_train_state* st) {
  if (!plan || !st) return fail(MPG_ERR_INVALID_ARG, "mpg_train_init: NULL argument");
  if (!(plan->budget > 0.0) || !(plan->train_fraction >= 0.0 && plan->train_fraction <= 1.0) ||
      plan->base_samples < 1)
    return fail(MPG_ERR_INVALID_ARG, "mpg_train_init: budget, training fraction or base sample count out of range");
  st->phase = plan->train_fraction > 0.0 ? MPG_TRAIN : MPG_RENDER;
  st->iteration = 0;
  st->target = plan->base_samples;
  st->done = 0;
  st->refit = 0;
  return MPG_OK;
}

extern "C" mpg_status mpg_train_step(const mpg_train_plan* plan, mpg_train_state* st, int64_t batch, double elapsed) {
  if (!plan || !st) return fail(MPG_ERR_INVALID_ARG, "mpg_train_step: NULL argument");
  if (batch < 0 || !(elapsed >= 0.0)) return fail(MPG_ERR_INVALID_ARG, "mpg_train_step: negative batch or time");
  st->refit = 0;
  if (st->phase != MPG_TRAIN) return MPG_OK;
  st->done += batch;
  const double train_budget = plan->train_fraction * plan->budget;
  if (elapsed >= train_budget) {
    // training ends now; the current iteration's samples make the guide
    st->phase = MPG_RENDER;
    st->refit = 1;
    return MPG_OK;
  }
  if (st->done >= st->target && elapsed < 0.5 * train_budget) {
    // iteration finished early enough: fit from it and double the next one
    st->refit = 1;
    st->iteration += 1;
    st->target *= 2;
    st->done = 0;
  }
  return MPG_OK;
}
