// Device code of both projectors.
#pragma once

#include "back_body.h"
#include "fwd_body.h"
