// internal.h -- declarations shared by the library's sources (not part of the
// C ABI).
#pragma once

#include "ai.h"

// Validate one request as ai_integrate validates its arguments: AI_OK,
// AI_WRTOL (rtol below 100 eps will be raised) or a negative ai_rc with the
// text in ai_last_error().
int ai_check_request(const ai_batch_item* item, int32_t kernel);

// Set the calling thread's ai_last_error() text and return rc.
int ai_fail(int rc, const char* msg);
